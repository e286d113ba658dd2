/*
 * Serial FP64 CPU oracle of the moist anelastic LES time step of
 * Chammas et al. (arXiv 2301.04698), Sec. 2 and App. A.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the GPU library.  Shares no
 * code with it.  Plain loops over cells; ghost cells are produced on demand
 * by at() so that every stencil below reads as it is written in the paper.
 *
 * Choices where the paper is silent are marked READING and listed with
 * their justification in the design notes of the repository.
 */
#include "les_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------ grid */

static size_t ncell(const ocfg *c) { return (size_t)c->nx * c->ny * c->nz; }

static size_t id3(const ocfg *c, int i, int j, int k) {
  return (size_t)i + (size_t)c->nx * ((size_t)j + (size_t)c->ny * (size_t)k);
}

static int wrapi(int i, int n) {
  while (i < 0) i += n;
  while (i >= n) i -= n;
  return i;
}

/* Cell value including ghost cells.  READING (boundary conditions):
 * x and y are periodic; across the rigid walls at z = 0 and z = H the ghost
 * mirrors the interior (k = -1 -> 0, k = -2 -> 1, k = nz -> nz-1, ...) times
 * `parity`: +1 for scalars, pressure, viscosity and buoyancy (zero normal
 * gradient: homogeneous Neumann, Sec. 2.4), -1 for w (zero wall mass flux)
 * and, with no-slip walls, for u and v (the paper's lid is no-slip and
 * zero-flux, Sec. 4, the surface is treated the same way); with free-slip
 * walls u and v are even (zero wall stress), see vpar. */
static double at(const ocfg *c, const double *f, int i, int j, int k, double parity) {
  i = wrapi(i, c->nx);
  j = wrapi(j, c->ny);
  if (k < 0) return parity * f[id3(c, i, j, -1 - k)];
  if (k >= c->nz) return parity * f[id3(c, i, j, 2 * c->nz - 1 - k)];
  return f[id3(c, i, j, k)];
}

/* Vertical profile value with even extension into the ghost levels. */
static double prof(const ocfg *c, const double *a, int k) {
  if (k < 0) k = -1 - k;
  if (k >= c->nz) k = 2 * c->nz - 1 - k;
  return a[k];
}

static const int UNIT[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* Wall parity of velocity component a.  READING (validation cases, Sec. 3):
 * the density current and rising bubble keep the free-slip rigid walls of
 * their original definitions (the paper replaces only the horizontal
 * boundaries by periodic ones), so u and v mirror evenly there; w is odd
 * under either condition. */
static double vpar(const ocfg *c, int a) { return a < 2 && c->wall == 1 ? 1.0 : -1.0; }

static double spacing(const ocfg *c, int axis) {
  return axis == 0 ? c->dx : (axis == 1 ? c->dy : c->dz);
}

static int check_cfg(const ocfg *c) {
  if (!c || c->nx < 1 || c->ny < 1 || c->nz < 4) return -1;
  if (!(c->dx > 0) || !(c->dy > 0) || !(c->dz > 0) || !(c->dt > 0)) return -1;
  if (c->advection != 0 && c->advection != 1) return -1;
  if (c->wall != 0 && c->wall != 1) return -1;
  if (!(c->nu_const >= 0.0) || c->nu_const > 1e6) return -1;
  if (c->phase != 0 && c->phase != 1) return -1;
  if (c->phase == 1 && !(c->T_ice > 0.0 && c->T_ice < c->Tf)) return -1;
  return 0;
}

/* ------------------------------------------------------ reference state */

typedef struct oprof {
  double *z, *p0, *T0, *rho0, *alpha0, *beta, *wsub;
} oprof;

/* Adiabatic hydrostatic reference state (Sec. 2.1, reference-state
 * equations): p0 = p00 (1 - g z / (cpd theta0))^(cpd/Rd),
 * T0 = theta0 (p0/p00)^(Rd/cpd), rho0 = p0 / (Rd T0), alpha0 = 1/rho0.
 * alpha0 is evaluated as Rd T0 / p0 (the same value as 1/rho0 written as the
 * equation of state alpha = R T / p0) so a dry state at theta_l = theta0 has
 * buoyancy exactly zero. */
int oracle_reference_state(const ocfg *c, double *p0, double *T0, double *rho0,
                           double *alpha0) {
  if (check_cfg(c)) return -1;
  for (int k = 0; k < c->nz; ++k) {
    double z = (k + 0.5) * c->dz; /* collocated cell centres */
    double pk = c->p00 * pow(1.0 - c->g * z / (c->cpd * c->theta0), c->cpd / c->Rd);
    double Tk = c->theta0 * pow(pk / c->p00, c->Rd / c->cpd);
    if (p0) p0[k] = pk;
    if (T0) T0[k] = Tk;
    if (rho0) rho0[k] = pk / (c->Rd * Tk);
    if (alpha0) alpha0[k] = c->Rd * Tk / pk;
  }
  return 0;
}

static void prof_free(oprof *P) {
  free(P->z); free(P->p0); free(P->T0); free(P->rho0); free(P->alpha0);
  free(P->beta); free(P->wsub);
}

static int prof_make(const ocfg *c, oprof *P) {
  int nz = c->nz;
  P->z = malloc(nz * sizeof(double));
  P->p0 = malloc(nz * sizeof(double));
  P->T0 = malloc(nz * sizeof(double));
  P->rho0 = malloc(nz * sizeof(double));
  P->alpha0 = malloc(nz * sizeof(double));
  P->beta = malloc(nz * sizeof(double));
  P->wsub = malloc(nz * sizeof(double));
  if (!P->z || !P->p0 || !P->T0 || !P->rho0 || !P->alpha0 || !P->beta || !P->wsub) {
    prof_free(P);
    return -1;
  }
  oracle_reference_state(c, P->p0, P->T0, P->rho0, P->alpha0);
  double H = nz * c->dz;
  double zs = (1.0 - c->sponge_frac) * H;
  for (int k = 0; k < nz; ++k) {
    double z = (k + 0.5) * c->dz;
    P->z[k] = z;
    /* READING (sponge, Sec. 2.3): linear Rayleigh damping in the top
     * sponge_frac of the domain with a sin^2 onset reaching sponge_max at
     * z = H. */
    double s = 0.0;
    if (z >= zs && H > zs) {
      double x = sin(0.5 * PI * (z - zs) / (H - zs));
      s = c->sponge_max * x * x;
    }
    P->beta[k] = s;
    /* READING (subsidence): w_sub = D z is the downward large-scale speed. */
    P->wsub[k] = c->wsub_div * z;
  }
  return 0;
}

/* ------------------------------------------------------ thermodynamics */

/* Exner function with the moist exponent R_m / c_pm (Sec. 2.1). */
double oracle_exner(const ocfg *c, double p0, double qt, double ql, double qi) {
  double qc = ql + qi;
  double Rm = (1.0 - qt) * c->Rd + (qt - qc) * c->Rv;
  double cpm = (1.0 - qt) * c->cpd + (qt - qc) * c->cpv + ql * c->cl + qi * c->ci;
  return pow(p0 / c->p00, Rm / cpm);
}

/* Liquid-ice potential temperature theta_l(T, q_l, q_i; p0) (Sec. 2.1). */
double oracle_theta_l(const ocfg *c, double T, double ql, double qi, double qt, double p0) {
  double qc = ql + qi;
  double cpm = (1.0 - qt) * c->cpd + (qt - qc) * c->cpv + ql * c->cl + qi * c->ci;
  double Pi = oracle_exner(c, p0, qt, ql, qi);
  return T / Pi * (1.0 - (c->Lv0 * ql + c->Ls0 * qi) / (cpm * T));
}

/* Saturation specific humidity.  READING (the paper defers the formula to
 * another reference): Clausius-Clapeyron with the constant latent heat L_v0
 * of Table 1 anchored at the triple point,
 *   e*(T) = e_tr exp[(L_v0/R_v)(1/T_tr - 1/T)],
 *   q_v*  = eps e* / (p0 - (1 - eps) e*),  eps = R_d / R_v. */
double oracle_qv_sat(const ocfg *c, double T, double p0) {
  double es = c->e_tr * exp(c->Lv0 / c->Rv * (1.0 / c->T_tr - 1.0 / T));
  double eps = c->Rd / c->Rv;
  return eps * es / (p0 - (1.0 - eps) * es);
}

/* Saturation specific humidity over ice: the same form with the
 * sublimation heat L_s0 of Table 1 (READING: the ice phase of Sec. 2.2
 * saturates over ice), equal to the liquid value at the triple point. */
double oracle_qv_sat_ice(const ocfg *c, double T, double p0) {
  double es = c->e_tr * exp(c->Ls0 / c->Rv * (1.0 / c->T_tr - 1.0 / T));
  double eps = c->Rd / c->Rv;
  return eps * es / (p0 - (1.0 - eps) * es);
}

/* Share lambda(T) of the condensate that is liquid.  Phase 0: the
 * Heaviside function of Sec. 2.2, H(T - T_f) with H(0) = 1.  Phase 1: the
 * continuous partition the paper suggests for mixed-phase clouds;
 * READING: the linear ramp of Tao et al. (1989), lambda = (T - T_ice) /
 * (T_f - T_ice) clipped to [0, 1]. */
double oracle_liquid_fraction(const ocfg *c, double T) {
  if (c->phase == 0) return T >= c->Tf ? 1.0 : 0.0;
  double lam = (T - c->T_ice) / (c->Tf - c->T_ice);
  return lam < 0.0 ? 0.0 : (lam > 1.0 ? 1.0 : lam);
}

/* Saturation humidity of the partitioned condensate (READING, after Tao
 * et al. 1989): lambda q_v*(liquid) + (1 - lambda) q_v*(ice). */
double oracle_qv_star(const ocfg *c, double T, double p0) {
  double lam = oracle_liquid_fraction(c, T);
  return lam * oracle_qv_sat(c, T, p0) + (1.0 - lam) * oracle_qv_sat_ice(c, T, p0);
}

/* Saturation partition at temperature T: q_c = max(0, q_t - q_v*),
 * q_l = lambda q_c, q_i = (1 - lambda) q_c (Sec. 2.2 with lambda in place of
 * the Heaviside functions). */
static void partition(const ocfg *c, double T, double qt, double p0, double *ql, double *qi) {
  double qc = fmax(0.0, qt - oracle_qv_star(c, T, p0));
  double lam = oracle_liquid_fraction(c, T);
  *ql = lam * qc;
  *qi = qc - *ql;
}

/* theta_l*(T; p0) - theta_l: the saturation-adjustment residual (Sec. 2.2). */
static double satadj_residual(const ocfg *c, double T, double thl, double qt, double p0) {
  double ql, qi;
  partition(c, T, qt, p0, &ql, &qi);
  return oracle_theta_l(c, T, ql, qi, qt, p0) - thl;
}

/* Saturation adjustment (Sec. 2.2): solve theta_l*(T) = theta_l by the
 * secant method.  READING: test the unsaturated temperature
 * T_u = theta_l Pi(q_c = 0) first; if q_t <= q_v*(T_u) it is the root.
 * Otherwise iterate from T_a = T_u and T_b = T_u + L_v0 (q_t - q_v*(T_u))/c_pd
 * until |T_b - T_a| <= satadj_tol, the two residuals coincide, or
 * satadj_maxit iterations.  Returns the number of secant iterations. */
int oracle_satadj(const ocfg *c, double thl, double qt, double p0, double *T, double *ql,
                  double *qi) {
  double Tu = thl * oracle_exner(c, p0, qt, 0.0, 0.0);
  double qs = oracle_qv_star(c, Tu, p0);
  if (qt <= qs) {
    *T = Tu; *ql = 0.0; *qi = 0.0;
    return 0;
  }
  double Ta = Tu, Tb = Tu + c->Lv0 * (qt - qs) / c->cpd;
  double fa = satadj_residual(c, Ta, thl, qt, p0);
  double fb = satadj_residual(c, Tb, thl, qt, p0);
  int it = 0;
  while (it < c->satadj_maxit) {
    if (fb == fa) break;
    double Tc = Tb - fb * (Tb - Ta) / (fb - fa);
    Ta = Tb; fa = fb;
    Tb = Tc; fb = satadj_residual(c, Tb, thl, qt, p0);
    ++it;
    if (fabs(Tb - Ta) <= c->satadj_tol) break;
  }
  *T = Tb;
  partition(c, Tb, qt, p0, ql, qi);
  return it;
}

/* Thermodynamic state of every cell; b = g (alpha - alpha0)/alpha0 with
 * alpha = R_m T / p0 (Sec. 2.1, buoyancy and equation of state). */
int oracle_thermo(const ocfg *c, const double *thl, const double *qt, double *T, double *ql,
                  double *qi, double *b) {
  if (check_cfg(c)) return -1;
  oprof P;
  if (prof_make(c, &P)) return -1;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        size_t n = id3(c, i, j, k);
        double Tc, qlc, qic;
        oracle_satadj(c, thl[n], qt[n], P.p0[k], &Tc, &qlc, &qic);
        double Rm = (1.0 - qt[n]) * c->Rd + (qt[n] - qlc - qic) * c->Rv;
        double alpha = Rm * Tc / P.p0[k];
        if (T) T[n] = Tc;
        if (ql) ql[n] = qlc;
        if (qi) qi[n] = qic;
        if (b) b[n] = c->g * (alpha - P.alpha0[k]) / P.alpha0[k];
      }
  prof_free(&P);
  return 0;
}

/* c_pm * Pi of a cell after saturation adjustment (radiative heating). */
static double cpm_pi(const ocfg *c, double qt, double ql, double qi, double p0) {
  double qc = ql + qi;
  double cpm = (1.0 - qt) * c->cpd + (qt - qc) * c->cpv + ql * c->cl + qi * c->ci;
  return cpm * oracle_exner(c, p0, qt, ql, qi);
}

/* ---------------------------------------------------------- SGS model */

/* Velocity gradient G[a][b] = d u_a / d x_b by central differences at a
 * cell (which may be a ghost cell). */
static void grad_u(const ocfg *c, const double *u, const double *v, const double *w, int i,
                   int j, int k, double G[3][3]) {
  const double *vel[3] = {u, v, w};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int *e = UNIT[b];
      double up = at(c, vel[a], i + e[0], j + e[1], k + e[2], vpar(c, a));
      double dn = at(c, vel[a], i - e[0], j - e[1], k - e[2], vpar(c, a));
      G[a][b] = (up - dn) / (2.0 * spacing(c, b));
    }
}

/* Smagorinsky-Lilly viscosity nu_t = (c_s Delta)^2 f_B S (Sec. 2.3) with
 * Delta = (dx dy dz)^(1/3).  READING: S = sqrt(2 S_ij S_ij); the buoyancy
 * factor is f_B = sqrt(clamp(1 - N^2 / (Pr S^2), 0, 1)) with
 * N^2 = d b / d z (central), and nu_t = 0 where S = 0.
 * The validation cases (Sec. 3) replace the model by a uniform kinematic
 * viscosity: nu = nu_const everywhere when nu_const > 0 (scalars then
 * diffuse with nu/Pr and nu/Sc like any other viscosity). */
int oracle_sgs_nu(const ocfg *c, const double *u, const double *v, const double *w,
                  const double *b, double *nu) {
  if (check_cfg(c)) return -1;
  if (c->nu_const > 0.0) {
    for (size_t q = 0; q < ncell(c); ++q) nu[q] = c->nu_const;
    return 0;
  }
  double delta = cbrt(c->dx * c->dy * c->dz);
  double l2 = (c->cs * delta) * (c->cs * delta);
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double G[3][3];
        grad_u(c, u, v, w, i, j, k, G);
        double S2 = 0.0;
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) {
            double s = 0.5 * (G[a][bb] + G[bb][a]);
            S2 += 2.0 * s * s;
          }
        double N2 = (at(c, b, i, j, k + 1, 1.0) - at(c, b, i, j, k - 1, 1.0)) / (2.0 * c->dz);
        double val = 0.0;
        if (S2 > 0.0) {
          double r = 1.0 - N2 / (c->Pr * S2);
          r = r < 0.0 ? 0.0 : (r > 1.0 ? 1.0 : r);
          val = l2 * sqrt(S2) * sqrt(r);
        }
        nu[id3(c, i, j, k)] = val;
      }
  return 0;
}

/* ----------------------------------------------------------- advection */

/* QUICK face value (Sec. 2.4; READING: Leonard's quadratic upstream
 * interpolation) at face l+1/2 from q at l-1 .. l+2, upwinded on the face
 * mass flux m. */
static double quick_face(double m, double qm1, double q0, double q1, double q2) {
  if (m >= 0.0) return (6.0 * q0 + 3.0 * q1 - qm1) / 8.0;
  return (6.0 * q1 + 3.0 * q0 - q2) / 8.0;
}

/* Third-order WENO reconstruction at face l+1/2 from the upwind side
 * (Sec. 3 alternative scheme; READING: the finite-volume WENO3 of Jiang &
 * Shu): a = q_{l-1}, b = q_l, c = q_{l+1}; candidates (-a + 3b)/2 on
 * {l-1, l} and (b + c)/2 on {l, l+1} with linear weights 1/3, 2/3;
 * smoothness (b - a)^2, (c - b)^2; eps = 1e-6 max(a^2, b^2, c^2) + 1e-18 so
 * the weights do not depend on the field's units. */
static double weno3_face(double a, double b, double c) {
  const double eps = 1e-6 * fmax(a * a, fmax(b * b, c * c)) + 1e-18;
  const double s0 = (eps + (b - a) * (b - a)), s1 = (eps + (c - b) * (c - b));
  /* w0 = (1/3)/s0^2 / ((1/3)/s0^2 + (2/3)/s1^2), written without the small squares
     in denominators */
  const double w0 = (1.0 / 3.0) * s1 * s1 / ((1.0 / 3.0) * s1 * s1 + (2.0 / 3.0) * s0 * s0);
  return w0 * (-a + 3.0 * b) / 2.0 + (1.0 - w0) * (b + c) / 2.0;
}

double oracle_face_value(int scheme, double qm1, double q0, double q1) {
  if (scheme == 1) return weno3_face(qm1, q0, q1);
  return (6.0 * q0 + 3.0 * q1 - qm1) / 8.0;
}

/* Advective flux through the face between a cell and its +1 neighbour along
 * `axis`: face mass flux m = (M_l + M_{l+1}) / 2 of the momentum component
 * along the axis, times the face value of q.  WENO3: Lax-Friedrichs flux
 * (1/2) m (q- + q+) - (1/2) |m| (q+ - q-) (READING: the local speed is |m|,
 * so the flux takes the reconstruction from the upwind side and vanishes
 * on the walls with m). */
static double adv_flux(const ocfg *c, const double *M, const double *q, double qpar, int axis,
                       int i, int j, int k) {
  const int *e = UNIT[axis];
  double m = 0.5 * (at(c, M, i, j, k, -1.0) + at(c, M, i + e[0], j + e[1], k + e[2], -1.0));
  double qm1 = at(c, q, i - e[0], j - e[1], k - e[2], qpar), q0 = at(c, q, i, j, k, qpar);
  double q1 = at(c, q, i + e[0], j + e[1], k + e[2], qpar);
  double q2 = at(c, q, i + 2 * e[0], j + 2 * e[1], k + 2 * e[2], qpar);
  if (c->advection == 1) {
    double qminus = weno3_face(qm1, q0, q1), qplus = weno3_face(q2, q1, q0);
    return 0.5 * m * (qminus + qplus) - 0.5 * fabs(m) * (qplus - qminus);
  }
  return m * quick_face(m, qm1, q0, q1, q2);
}

/* out = -div(U q) in flux form (Sec. 2.1 conservation form) with QUICK
 * (Sec. 2.4) or WENO3/Lax-Friedrichs face fluxes.  U, V, W are momentum
 * components rho0 u. */
int oracle_advect(const ocfg *c, const double *U, const double *V, const double *W,
                  const double *q, double zparity, double *out) {
  if (check_cfg(c)) return -1;
  const double *M[3] = {U, V, W};
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int *e = UNIT[a];
          double fp = adv_flux(c, M[a], q, zparity, a, i, j, k);
          double fm = adv_flux(c, M[a], q, zparity, a, i - e[0], j - e[1], k - e[2]);
          s -= (fp - fm) / spacing(c, a);
        }
        out[id3(c, i, j, k)] = s;
      }
  return 0;
}

/* ----------------------------------------------------------- diffusion */

/* out = div(rho0 nu/Pr grad q): 2nd-order central diffusion in face form
 * (Sec. 2.4).  READING: face viscosity is the mean of the two cells, the
 * vertical face rho0 the mean of the two levels. */
int oracle_diffuse(const ocfg *c, const double *nu, double inv_prandtl, const double *q,
                   double *out) {
  if (check_cfg(c)) return -1;
  oprof P;
  if (prof_make(c, &P)) return -1;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int *e = UNIT[a];
          double d = spacing(c, a);
          double F[2];
          for (int side = 0; side < 2; ++side) {
            /* face between cell l = (i,j,k) - side*e and l + e */
            int li = i - side * e[0], lj = j - side * e[1], lk = k - side * e[2];
            double nuf = 0.5 * (at(c, nu, li, lj, lk, 1.0) +
                                at(c, nu, li + e[0], lj + e[1], lk + e[2], 1.0));
            double rf = a == 2 ? 0.5 * (prof(c, P.rho0, lk) + prof(c, P.rho0, lk + 1)) : P.rho0[k];
            double g = (at(c, q, li + e[0], lj + e[1], lk + e[2], 1.0) - at(c, q, li, lj, lk, 1.0)) / d;
            F[side] = rf * nuf * inv_prandtl * g;
          }
          s += (F[0] - F[1]) / d;
        }
        out[id3(c, i, j, k)] = s;
      }
  prof_free(&P);
  return 0;
}

/* div(rho0 sigma) with sigma_ij = nu (d_i u_j + d_j u_i) (Sec. 2.3).
 * READING: on the face normal to axis i the compact difference gives
 * d_i u_j and the mean of the two cell-centred central differences gives
 * d_j u_i; face viscosity and rho0 as in oracle_diffuse. */
int oracle_sgs_momentum(const ocfg *c, const double *nu, const double *u, const double *v,
                        const double *w, double *fx, double *fy, double *fz) {
  if (check_cfg(c)) return -1;
  oprof P;
  if (prof_make(c, &P)) return -1;
  const double *vel[3] = {u, v, w};
  double *out[3] = {fx, fy, fz};
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double div[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < 3; ++ax) {
          const int *e = UNIT[ax];
          double d = spacing(c, ax);
          double F[2][3];
          for (int side = 0; side < 2; ++side) {
            int li = i - side * e[0], lj = j - side * e[1], lk = k - side * e[2];
            int ri = li + e[0], rj = lj + e[1], rk = lk + e[2];
            double Gl[3][3], Gr[3][3];
            grad_u(c, u, v, w, li, lj, lk, Gl);
            grad_u(c, u, v, w, ri, rj, rk, Gr);
            double nuf = 0.5 * (at(c, nu, li, lj, lk, 1.0) + at(c, nu, ri, rj, rk, 1.0));
            double rf = ax == 2 ? 0.5 * (prof(c, P.rho0, lk) + prof(c, P.rho0, rk)) : P.rho0[k];
            for (int comp = 0; comp < 3; ++comp) {
              double dij = (at(c, vel[comp], ri, rj, rk, vpar(c, comp)) -
                            at(c, vel[comp], li, lj, lk, vpar(c, comp))) / d;
              double dji = 0.5 * (Gl[ax][comp] + Gr[ax][comp]);
              F[side][comp] = rf * nuf * (dij + dji);
            }
          }
          for (int comp = 0; comp < 3; ++comp) div[comp] += (F[0][comp] - F[1][comp]) / d;
        }
        size_t n = id3(c, i, j, k);
        for (int comp = 0; comp < 3; ++comp) out[comp][n] = div[comp];
      }
  prof_free(&P);
  return 0;
}

/* ------------------------------------------------- discrete operators */

/* Compact 7-point Laplacian (App. A, second-difference operator); even
 * mirror across the walls = homogeneous Neumann (Sec. 2.4). */
int oracle_laplacian(const ocfg *c, const double *phi, double *out) {
  if (check_cfg(c)) return -1;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int *e = UNIT[a];
          double d = spacing(c, a);
          s += (at(c, phi, i + e[0], j + e[1], k + e[2], 1.0) - 2.0 * at(c, phi, i, j, k, 1.0) +
                at(c, phi, i - e[0], j - e[1], k - e[2], 1.0)) / (d * d);
        }
        out[id3(c, i, j, k)] = s;
      }
  return 0;
}

/* Collocated-grid consistency correction C of App. A: the wide operator
 * div_c grad_c minus the compact Laplacian, i.e. per axis
 * (q_{l+2} - 4 q_{l+1} + 6 q_l - 4 q_{l-1} + q_{l-2}) / (4 Delta^2). */
int oracle_app_a(const ocfg *c, const double *phi, double *out) {
  if (check_cfg(c)) return -1;
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int *e = UNIT[a];
          double d = spacing(c, a);
          double q2p = at(c, phi, i + 2 * e[0], j + 2 * e[1], k + 2 * e[2], 1.0);
          double q1p = at(c, phi, i + e[0], j + e[1], k + e[2], 1.0);
          double q0 = at(c, phi, i, j, k, 1.0);
          double q1m = at(c, phi, i - e[0], j - e[1], k - e[2], 1.0);
          double q2m = at(c, phi, i - 2 * e[0], j - 2 * e[1], k - 2 * e[2], 1.0);
          s += (q2p - 4.0 * q1p + 6.0 * q0 - 4.0 * q1m + q2m) / (4.0 * d * d);
        }
        out[id3(c, i, j, k)] = s;
      }
  return 0;
}

/* Central divergence div_c (App. A, first-difference operator). */
int oracle_divergence(const ocfg *c, const double *U, const double *V, const double *W,
                      double *out) {
  if (check_cfg(c)) return -1;
  const double *M[3] = {U, V, W};
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a) {
          const int *e = UNIT[a];
          s += (at(c, M[a], i + e[0], j + e[1], k + e[2], -1.0) -
                at(c, M[a], i - e[0], j - e[1], k - e[2], -1.0)) / (2.0 * spacing(c, a));
        }
        out[id3(c, i, j, k)] = s;
      }
  return 0;
}

/* Radiative heating -(c_pm Pi)^-1 d(rho0 F_R)/dz (Sec. 2.1, theta_l
 * equation).  READING (synthetic longwave flux standing in for the case's
 * own formula): net upward flux at face height z_f is
 * F0 exp(-kappa * sum over cells above z_f of rho0 q_l dz). */
int oracle_radiation(const ocfg *c, const double *ql, const double *cpmpi, double *out) {
  if (check_cfg(c)) return -1;
  oprof P;
  if (prof_make(c, &P)) return -1;
  double *F = malloc((c->nz + 1) * sizeof(double));
  if (!F) { prof_free(&P); return -1; }
  for (int j = 0; j < c->ny; ++j)
    for (int i = 0; i < c->nx; ++i) {
      double lwp = 0.0;
      F[c->nz] = c->rad_F0;
      for (int k = c->nz - 1; k >= 0; --k) {
        lwp += P.rho0[k] * ql[id3(c, i, j, k)] * c->dz;
        F[k] = c->rad_F0 * exp(-c->rad_kappa * lwp);
      }
      for (int k = 0; k < c->nz; ++k) {
        size_t n = id3(c, i, j, k);
        out[n] = -(F[k + 1] - F[k]) / (c->dz * cpmpi[n]);
      }
    }
  free(F);
  prof_free(&P);
  return 0;
}

/* ---------------------------------------------------------- reductions */

static double fsum(const ocfg *c, const double *f) {
  double s = 0.0;
  size_t n = ncell(c);
  for (size_t q = 0; q < n; ++q) s += f[q];
  return s;
}

static double fnorm2(const ocfg *c, const double *f) {
  double s = 0.0;
  size_t n = ncell(c);
  for (size_t q = 0; q < n; ++q) s += f[q] * f[q];
  return sqrt(s);
}

/* -------------------------------------------------------- Poisson solve */

/* Neighbour indices of row/column l on a periodic axis of length n. */
static void periodic_nb(int l, int n, int *lm, int *lp) {
  *lm = l == 0 ? n - 1 : l - 1;
  *lp = l == n - 1 ? 0 : l + 1;
}

/* Sum over axes of (phi_+ + phi_-) / Delta^2 for every cell: the
 * off-diagonal part of the compact Laplacian.  z neighbours across a wall
 * are the even-mirror ghosts (k = -1 -> 0, k = nz -> nz-1). */
static void neighbour_sum(const ocfg *c, const double *phi, double *nb) {
  double ix2 = 1.0 / (c->dx * c->dx), iy2 = 1.0 / (c->dy * c->dy), iz2 = 1.0 / (c->dz * c->dz);
  for (int k = 0; k < c->nz; ++k) {
    int km = k == 0 ? 0 : k - 1, kp = k == c->nz - 1 ? c->nz - 1 : k + 1;
    for (int j = 0; j < c->ny; ++j) {
      int jm, jp;
      periodic_nb(j, c->ny, &jm, &jp);
      for (int i = 0; i < c->nx; ++i) {
        int im, ip;
        periodic_nb(i, c->nx, &im, &ip);
        nb[id3(c, i, j, k)] = (phi[id3(c, ip, j, k)] + phi[id3(c, im, j, k)]) * ix2 +
                              (phi[id3(c, i, jp, k)] + phi[id3(c, i, jm, k)]) * iy2 +
                              (phi[id3(c, i, j, kp)] + phi[id3(c, i, j, km)]) * iz2;
      }
    }
  }
}

/* Extreme nonzero eigenvalues of -D^{-1} L for the compact Laplacian L with
 * periodic x, y and mirror-Neumann z, D = 2/dx^2 + 2/dy^2 + 2/dz^2:
 * periodic axis (2 - 2 cos(2 pi m / N)) / Delta^2, mirror axis
 * (2 - 2 cos(pi m / N)) / Delta^2, m = 0 .. N-1; an eigenvalue of L is the
 * sum over the axes.  A periodic axis of one cell has only its m = 0 mode
 * and no smallest nonzero eigenvalue.  With mean_mode 2 the sweeps act only
 * on modes with both horizontal (m_x or m_y > 0) and vertical (m_z > 0)
 * structure, whose smallest eigenvalue is the smallest horizontal one plus
 * the smallest vertical one. */
int oracle_jacobi_bounds(const ocfg *c, double *mu_min, double *mu_max) {
  if (check_cfg(c)) return -1;
  double d = 2.0 / (c->dx * c->dx) + 2.0 / (c->dy * c->dy) + 2.0 / (c->dz * c->dz);
  double lx1 = (2.0 - 2.0 * cos(2.0 * PI / c->nx)) / (c->dx * c->dx);
  double ly1 = (2.0 - 2.0 * cos(2.0 * PI / c->ny)) / (c->dy * c->dy);
  double lz1 = (2.0 - 2.0 * cos(PI / c->nz)) / (c->dz * c->dz);
  double lxm = (2.0 - 2.0 * cos(2.0 * PI * (c->nx / 2) / c->nx)) / (c->dx * c->dx);
  double lym = (2.0 - 2.0 * cos(2.0 * PI * (c->ny / 2) / c->ny)) / (c->dy * c->dy);
  double lzm = (2.0 - 2.0 * cos(PI * (c->nz - 1) / c->nz)) / (c->dz * c->dz);
  double mn = lz1, mh = 0.0;
  if (c->nx > 1) mh = lx1;
  if (c->ny > 1 && (mh == 0.0 || ly1 < mh)) mh = ly1;
  if (c->mean_mode == 2) {
    /* the sweeps see only modes with horizontal and vertical structure */
    mn = mh + lz1;
  } else if (mh > 0.0 && mh < mn) {
    mn = mh;
  }
  *mu_min = mn / d;
  *mu_max = (lxm + lym + lzm) / d;
  return 0;
}

/* Horizontal mean of field f on every level. */
static void level_means(const ocfg *c, const double *f, double *mean) {
  size_t nxy = (size_t)c->nx * c->ny;
  for (int k = 0; k < c->nz; ++k) {
    double s = 0.0;
    for (size_t q = 0; q < nxy; ++q) s += f[(size_t)k * nxy + q];
    mean[k] = s / (double)nxy;
  }
}

/* The horizontally uniform part of L phi = rhs.  READING (the paper sweeps
 * every mode): the compact Laplacian maps a function of z alone to its
 * second difference in z, and horizontal averaging commutes with it, so the
 * horizontal mean of the equation is the one-dimensional Neumann problem
 *   (pb_{k+1} - 2 pb_k + pb_{k-1}) / dz^2 = rb_k   (mirror ghosts),
 * decoupled from the other modes.  Its exact solution: the face gradient
 * G_{k+1/2} = (pb_{k+1} - pb_k)/dz is zero at the bottom wall and grows by
 * dz rb_k across level k, so G_{k+1/2} = dz sum_{m<=k} rb_m and
 * pb_{k+1} = pb_k + dz G_{k+1/2}; then the vertical mean is removed.  rb has
 * zero vertical mean (the rhs mean is removed), which is what makes the
 * gradient at the top wall vanish too. */
static void mean_mode_solve(const ocfg *c, const double *rb, double *pb) {
  double G = 0.0, s = 0.0;
  pb[0] = 0.0;
  for (int k = 0; k + 1 < c->nz; ++k) {
    G += c->dz * rb[k];
    pb[k + 1] = pb[k] + c->dz * G;
  }
  for (int k = 0; k < c->nz; ++k) s += pb[k];
  for (int k = 0; k < c->nz; ++k) pb[k] -= s / c->nz;
}

/* Vertical mean of field f in every column (i, j): mean[i + nx j]. */
static void column_means(const ocfg *c, const double *f, double *mean) {
  size_t nxy = (size_t)c->nx * c->ny;
  for (size_t q = 0; q < nxy; ++q) {
    double s = 0.0;
    for (int k = 0; k < c->nz; ++k) s += f[(size_t)k * nxy + q];
    mean[q] = s / c->nz;
  }
}

/* cas(2 pi m / n) = cos + sin of the angle, m taken modulo n. */
static double cas_angle(long m, int n) {
  double t = 2.0 * PI * (double)(m % n) / n;
  return cos(t) + sin(t);
}

/* The vertically uniform part of L phi = rhs (mean_mode 2).  READING (the
 * paper sweeps every mode): with mirror walls the z second differences of a
 * column sum to zero, and the z part of L vanishes on a field constant in
 * z, so the vertical mean of the equation is the two-dimensional periodic
 * problem Lh pv = rv, Lh the x and y part of L, which decouples from the
 * modes with vertical structure.  Its exact solution in the real Fourier
 * (Hartley) basis, which diagonalises each periodic second difference:
 * with H[k][i] = cas(2 pi k i / n) (H H = n I) and the eigenvalue of mode
 * (kx, ky) lambda = -(2 - 2 cos(2 pi kx/nx))/dx^2 - (2 - 2 cos(2 pi ky/ny))/dy^2,
 *   pv = Hy [ (Hy rv Hx) / lambda ] Hx / (nx ny),
 * the mode (0, 0) (the mean, zero for a centred rhs) set to zero.  Plain
 * sums, O(nx ny (nx + ny)). */
static int vertical_mode_solve(const ocfg *c, const double *rv, double *pv) {
  int nx = c->nx, ny = c->ny;
  size_t nxy = (size_t)nx * ny;
  double *a = malloc(nxy * sizeof(double)), *b = malloc(nxy * sizeof(double));
  if (!a || !b) { free(a); free(b); return -1; }
  /* a = Hy rv: a[ky][i] = sum_j cas(2 pi ky j / ny) rv[j][i] */
  for (int ky = 0; ky < ny; ++ky)
    for (int i = 0; i < nx; ++i) {
      double s = 0.0;
      for (int j = 0; j < ny; ++j) s += cas_angle((long)ky * j, ny) * rv[(size_t)j * nx + i];
      a[(size_t)ky * nx + i] = s;
    }
  /* b = a Hx, divided by the eigenvalue */
  for (int ky = 0; ky < ny; ++ky)
    for (int kx = 0; kx < nx; ++kx) {
      double s = 0.0;
      for (int i = 0; i < nx; ++i) s += a[(size_t)ky * nx + i] * cas_angle((long)i * kx, nx);
      double lam = -(2.0 - 2.0 * cos(2.0 * PI * kx / nx)) / (c->dx * c->dx)
                   - (2.0 - 2.0 * cos(2.0 * PI * ky / ny)) / (c->dy * c->dy);
      b[(size_t)ky * nx + kx] = (kx == 0 && ky == 0) ? 0.0 : s / lam;
    }
  /* pv = Hy b Hx / (nx ny) */
  for (int j = 0; j < ny; ++j)
    for (int kx = 0; kx < nx; ++kx) {
      double s = 0.0;
      for (int ky = 0; ky < ny; ++ky) s += cas_angle((long)j * ky, ny) * b[(size_t)ky * nx + kx];
      a[(size_t)j * nx + kx] = s;
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      double s = 0.0;
      for (int kx = 0; kx < nx; ++kx) s += a[(size_t)j * nx + kx] * cas_angle((long)kx * i, nx);
      pv[(size_t)j * nx + i] = s / ((double)nx * ny);
    }
  free(a); free(b);
  return 0;
}

int oracle_vertical_mode_solve(const ocfg *c, const double *rv, double *pv) {
  if (check_cfg(c)) return -1;
  return vertical_mode_solve(c, rv, pv);
}

/* ||rhs - L phi||_2 with L phi = neighbour sum - D phi. */
static double residual_norm(const ocfg *c, const double *rhs, const double *phi, double *tmp) {
  double d = 2.0 / (c->dx * c->dx) + 2.0 / (c->dy * c->dy) + 2.0 / (c->dz * c->dz);
  neighbour_sum(c, phi, tmp);
  double s = 0.0;
  for (size_t q = 0; q < ncell(c); ++q) {
    double r = rhs[q] - (tmp[q] - d * phi[q]);
    s += r * r;
  }
  return sqrt(s);
}

/* Weighted-Jacobi sweeps on L phi = rhs (rhs centred) from the iterate in
 * phi until ||rhs - L phi||_2 <= tol * rn (checked every check_every
 * sweeps), the cap, or exactly fixed_sweeps sweeps:
 *   phi' = (1 - w) phi + w [sum_axes (phi_+ + phi_-)/Delta^2 - rhs] / D.
 * READING: w = 2 / (mu_min + mu_max) unless set; scheme 1 accelerates the
 * same sweep with the Chebyshev two-term recurrence
 *   phi_{m+1} = phi_{m-1} + w_{m+1} (J(phi_m) - phi_{m-1}),
 *   w_1 = 1, w_2 = 1/(1 - rho^2/2), w_{m+1} = 1/(1 - rho^2 w_m / 4),
 * rho = (mu_max - mu_min)/(mu_max + mu_min).  Returns the status (0
 * converged, 1 not converged, -3 non-finite); *sweeps and *res get the
 * sweep count and the residual norm of the returned iterate. */
static int jacobi_sweeps(const ocfg *c, const double *rhs, double rn, double *phi,
                         int32_t fixed_sweeps, double *tmp, double *prev, int *sweeps,
                         double *res) {
  size_t n = ncell(c);
  double d = 2.0 / (c->dx * c->dx) + 2.0 / (c->dy * c->dy) + 2.0 / (c->dz * c->dz);
  double mu0, mu1;
  oracle_jacobi_bounds(c, &mu0, &mu1);
  double omega = c->jacobi_omega > 0.0 ? c->jacobi_omega : 2.0 / (mu0 + mu1);
  double rho = (mu1 - mu0) / (mu1 + mu0);
  double wcheb = 1.0;
  memcpy(prev, phi, n * sizeof(double));
  int m = 0, status = 1;
  double rr = 0.0;
  for (;;) {
    int check = fixed_sweeps > 0 ? (m == fixed_sweeps)
                                 : (m % c->poisson_check_every == 0 || m >= c->poisson_max_sweeps);
    if (check) {
      rr = residual_norm(c, rhs, phi, tmp);
      if (!isfinite(rr)) { status = -3; break; }
      if (fixed_sweeps > 0) { status = rr <= c->poisson_tol * rn ? 0 : 1; break; }
      if (rr <= c->poisson_tol * rn) { status = 0; break; }
      if (m >= c->poisson_max_sweeps) { status = 1; break; }
    }
    /* one sweep: tmp = J(phi), the weighted-Jacobi update */
    double wj = c->poisson_scheme == 1 ? 2.0 / (mu0 + mu1) : omega;
    neighbour_sum(c, phi, tmp);
    for (size_t q = 0; q < n; ++q) tmp[q] = (1.0 - wj) * phi[q] + wj * (tmp[q] - rhs[q]) / d;
    if (c->poisson_scheme == 1) {
      if (m == 0) wcheb = 1.0;
      else if (m == 1) wcheb = 1.0 / (1.0 - 0.5 * rho * rho);
      else wcheb = 1.0 / (1.0 - 0.25 * rho * rho * wcheb);
      for (size_t q = 0; q < n; ++q) {
        double next = prev[q] + wcheb * (tmp[q] - prev[q]);
        prev[q] = phi[q];
        phi[q] = next;
      }
    } else {
      memcpy(phi, tmp, n * sizeof(double));
    }
    ++m;
  }
  *sweeps = m;
  *res = rr;
  return status;
}

/* Solve L phi = rhs (Sec. 2.4, pressure-correction equation; the unknown is
 * phi = alpha0 delta p).  rhs gets its mean removed (compatibility); the
 * stopping test is relative to its norm; the solution has zero mean.
 * The zero start is phi = 0, or with mean_mode >= 1 the exact solution of
 * the horizontally uniform part (mean_mode_solve), with mean_mode 2 plus
 * that of the vertically uniform part (vertical_mode_solve).  phi in holds
 * the guess: the start is the zero start plus the guess with those exact
 * parts removed (its horizontal means per level, and with mean_mode 2 its
 * vertical means per column, its overall mean added back).  With
 * mean_mode 2 the sweeps' correction is projected the same way at the end
 * (in exact arithmetic a no-op: the sweeps keep both parts of it zero) and
 * the residual reported is that of the returned iterate.  gate = 1: the guess is kept only if its residual is below the
 * zero start's, and a kept guess whose sweeps reach the cap (no fixed
 * count) is dropped and the sweeps repeated from the zero start.  budget >
 * 0 (no fixed count): a kept guess's sweeps stop at the first residual
 * check at or beyond `budget` sweeps, counting as reaching the cap (a
 * guess that needs more sweeps than the zero start did is no use). */
static int poisson_solve(const ocfg *c, const double *rhs_in, double *phi, int32_t fixed_sweeps,
                         int gate, int budget, osolve *st) {
  if (check_cfg(c)) return -1;
  size_t n = ncell(c), nxy = (size_t)c->nx * c->ny;
  double *rhs = malloc(n * sizeof(double));
  double *tmp = malloc(n * sizeof(double));
  double *prev = malloc(n * sizeof(double));
  double *zero = malloc(n * sizeof(double));
  double *rb = malloc(c->nz * sizeof(double));
  double *pb = malloc(c->nz * sizeof(double));
  double *gb = malloc(c->nz * sizeof(double));
  double *rv = calloc(nxy, sizeof(double));
  double *pv = calloc(nxy, sizeof(double));
  double *gv = calloc(nxy, sizeof(double));
  if (!rhs || !tmp || !prev || !zero || !rb || !pb || !gb || !rv || !pv || !gv) {
    free(rhs); free(tmp); free(prev); free(zero); free(rb); free(pb); free(gb);
    free(rv); free(pv); free(gv);
    return -1;
  }
  double mr = fsum(c, rhs_in) / (double)n;
  for (size_t q = 0; q < n; ++q) rhs[q] = rhs_in[q] - mr;
  double rn = fnorm2(c, rhs);
  /* zero start, and the guess without the parts that start exact */
  double gm = 0.0;
  for (int k = 0; k < c->nz; ++k) pb[k] = gb[k] = 0.0;
  if (c->mean_mode >= 1) {
    level_means(c, rhs, rb);
    mean_mode_solve(c, rb, pb);
    level_means(c, phi, gb);
  }
  if (c->mean_mode == 2) {
    column_means(c, rhs, rv);
    if (vertical_mode_solve(c, rv, pv)) {
      free(rhs); free(tmp); free(prev); free(zero); free(rb); free(pb); free(gb);
      free(rv); free(pv); free(gv);
      return -1;
    }
    column_means(c, phi, gv);
    gm = fsum(c, phi) / (double)n;
  }
  for (int k = 0; k < c->nz; ++k)
    for (size_t q = 0; q < nxy; ++q) {
      size_t qq = (size_t)k * nxy + q;
      zero[qq] = pb[k] + pv[q];
      phi[qq] = zero[qq] + (phi[qq] - gb[k] - gv[q] + gm);
    }
  int guessed = 0;
  if (gate) {
    guessed = 1;
    if (!(residual_norm(c, rhs, phi, tmp) < residual_norm(c, rhs, zero, tmp))) {
      memcpy(phi, zero, n * sizeof(double));
      guessed = 2;
    }
  }
  /* the sweeps' start (mean_mode 2 projects the correction against it) */
  double *start = NULL;
  if (c->mean_mode == 2) {
    start = malloc(n * sizeof(double));
    if (!start) {
      free(rhs); free(tmp); free(prev); free(zero); free(rb); free(pb); free(gb);
      free(rv); free(pv); free(gv);
      return -1;
    }
    memcpy(start, phi, n * sizeof(double));
  }
  int m = 0, status = 0, first = 0;
  double rr = 0.0;
  if (rn > 0.0) {
    ocfg cb = *c; /* a kept guess's sweeps end at the first check from `budget` on */
    if (guessed == 1 && fixed_sweeps == 0 && budget > 0) {
      int b = (budget + c->poisson_check_every - 1) / c->poisson_check_every * c->poisson_check_every;
      if (b < cb.poisson_max_sweeps) cb.poisson_max_sweeps = b;
    }
    status = jacobi_sweeps(&cb, rhs, rn, phi, fixed_sweeps, tmp, prev, &m, &rr);
    if (status == 1 && guessed == 1 && fixed_sweeps == 0) {
      int m2 = 0;
      memcpy(phi, zero, n * sizeof(double));
      if (start) memcpy(start, zero, n * sizeof(double));
      status = jacobi_sweeps(c, rhs, rn, phi, 0, tmp, prev, &m2, &rr);
      first = m;
      m += m2;
      guessed = 3;
    }
  }
  if (c->mean_mode == 2 && rn > 0.0) {
    /* the correction relative to the last pass's start, without the parts
       that started exact (each zero in exact arithmetic) */
    for (size_t q = 0; q < n; ++q) tmp[q] = phi[q] - start[q];
    level_means(c, tmp, gb);
    column_means(c, tmp, gv);
    double dm = fsum(c, tmp) / (double)n;
    for (int k = 0; k < c->nz; ++k)
      for (size_t q = 0; q < nxy; ++q) {
        size_t qq = (size_t)k * nxy + q;
        phi[qq] = start[qq] + (tmp[qq] - gb[k] - gv[q] + dm);
      }
    rr = residual_norm(c, rhs, phi, tmp);
  }
  double mp = fsum(c, phi) / (double)n;
  for (size_t q = 0; q < n; ++q) phi[q] -= mp;
  if (st) {
    st->sweeps = m;
    st->status = status;
    st->rhs_norm = rn;
    st->res_norm = rr;
    st->guess = guessed;
    st->guess_sweeps = first;
  }
  free(rhs); free(tmp); free(prev); free(zero); free(rb); free(pb); free(gb);
  free(rv); free(pv); free(gv); free(start);
  return status < 0 ? status : 0;
}

int oracle_poisson(const ocfg *c, const double *rhs_in, double *phi, int32_t fixed_sweeps,
                   osolve *st) {
  return poisson_solve(c, rhs_in, phi, fixed_sweeps, 0, 0, st);
}

int oracle_poisson_gated(const ocfg *c, const double *rhs_in, double *phi, int32_t fixed_sweeps,
                         int32_t budget, osolve *st) {
  return poisson_solve(c, rhs_in, phi, fixed_sweeps, 1, budget, st);
}

/* ---------------------------------------------------------- time step */

typedef struct ostate {
  double *Un[3], *Uk[3], *Uh[3], *uh[3], *uk[3], *Uhat[3], *R[3], *sg[3];
  double *thl_h, *qt_h, *thl_m, *qt_m, *b_h, *b_m, *ql_m, *qi_m, *cpmpi_m;
  double *nu_s, *nu_m, *tend, *tmp, *psi, *rhs, *phi, *phi_lag;
} ostate;

#define OS_NPTR ((int)(sizeof(ostate) / sizeof(double *)))

static void ostate_free(ostate *s) {
  double **p = (double **)s;
  for (int q = 0; q < OS_NPTR; ++q) free(p[q]);
}

static int ostate_alloc(ostate *s, size_t n) {
  memset(s, 0, sizeof(*s));
  double **p = (double **)s;
  for (int q = 0; q < OS_NPTR; ++q) {
    p[q] = calloc(n, sizeof(double));
    if (!p[q]) { ostate_free(s); return -1; }
  }
  return 0;
}

/* Scalar source terms other than advection and diffusion (Sec. 2.1 scalar
 * equations, READING of the forcing): subsidence rho0 w_sub d phi/dz,
 * surface flux into the lowest cell (sensible: SHF/c_pd for theta_l, latent:
 * LHF/L_v0 for q_t, per unit area, divided by dz). */
static void scalar_sources(const ocfg *c, const oprof *P, const double *phi, double sfc,
                           double *tend) {
  for (int k = 0; k < c->nz; ++k)
    for (int j = 0; j < c->ny; ++j)
      for (int i = 0; i < c->nx; ++i) {
        size_t n = id3(c, i, j, k);
        double dphi = (at(c, phi, i, j, k + 1, 1.0) - at(c, phi, i, j, k - 1, 1.0)) / (2.0 * c->dz);
        tend[n] += P->rho0[k] * P->wsub[k] * dphi;
        if (k == 0) tend[n] += sfc / c->dz;
      }
}

/* One or more time steps of the iterative predictor-corrector scheme
 * (Sec. 2.4): scalars advance from n+1/2 to n+3/2 with velocity u^k and
 * phi^{n+1} = (phi^k + phi^{n+1/2})/2; momentum is predicted with the
 * pressure of the previous sub-iteration and R^{n+1/2} from
 * (u^k + u^n)/2 and b^{n+1/2}, then projected by the pressure correction
 * solved from the Poisson equation with the App. A correction of the
 * previous sub-iteration's phi (zero at a step's start). */
int oracle_step(const ocfg *c, double *u, double *v, double *w, double *thl, double *qt,
                double *p, int32_t nsteps, const int32_t *replay, osolve *rec, odebug *dbg) {
  if (check_cfg(c) || c->n_subiter < 1 || c->guess < 0 || c->guess > 2) return -1;
  size_t n = ncell(c);
  oprof P;
  if (prof_make(c, &P)) return -1;
  ostate S;
  if (ostate_alloc(&S, n)) { prof_free(&P); return -1; }
  /* guess memory: the previous step's pressure, or one solution per sub-iteration */
  size_t nhist = c->guess == 1 ? n : c->guess == 2 ? (size_t)c->n_subiter * n : 0;
  double *hist = nhist ? calloc(nhist, sizeof(double)) : NULL;
  /* sweeps of the last solve of each sub-iteration that ran from the zero
     start: the budget of a kept guess (0: none yet) */
  int *zero_sweeps = calloc(c->n_subiter, sizeof(int));
  if (!zero_sweeps) { free(hist); ostate_free(&S); prof_free(&P); return -1; }
  if (nhist && !hist) { ostate_free(&S); prof_free(&P); return -1; }
  if (c->guess == 1) memcpy(hist, p, n * sizeof(double));
  double *vel[3] = {u, v, w};
  double ugv[3] = {c->ug, c->vg, 0.0};
  int solve = 0, rc = 0;

  for (int step = 0; step < nsteps && rc == 0; ++step) {
    /* U^n = rho0 u^n; Phi^{n+1/2}; b^{n+1/2} */
    for (int k = 0; k < c->nz; ++k)
      for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
        for (int a = 0; a < 3; ++a) {
          S.Un[a][q] = P.rho0[k] * vel[a][q];
          S.Uk[a][q] = S.Un[a][q];
        }
    memcpy(S.thl_h, thl, n * sizeof(double));
    memcpy(S.qt_h, qt, n * sizeof(double));
    oracle_thermo(c, S.thl_h, S.qt_h, NULL, NULL, NULL, S.b_h);
    memset(S.phi_lag, 0, n * sizeof(double));

    for (int it = 0; it < c->n_subiter && rc == 0; ++it) {
      /* --- scalars: Phi^{k+1} = Phi^{n+1/2} + dt/rho0 [ ... ](Phi_mid, U^k) */
      for (size_t q = 0; q < n; ++q) {
        S.thl_m[q] = 0.5 * (thl[q] + S.thl_h[q]);
        S.qt_m[q] = 0.5 * (qt[q] + S.qt_h[q]);
      }
      double *Tdummy = S.tmp;
      oracle_thermo(c, S.thl_m, S.qt_m, Tdummy, S.ql_m, S.qi_m, S.b_m);
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q) {
          S.cpmpi_m[q] = cpm_pi(c, S.qt_m[q], S.ql_m[q], S.qi_m[q], P.p0[k]);
          for (int a = 0; a < 3; ++a) S.uk[a][q] = S.Uk[a][q] / P.rho0[k];
        }
      oracle_sgs_nu(c, S.uk[0], S.uk[1], S.uk[2], S.b_m, S.nu_s);

      /* theta_l */
      oracle_advect(c, S.Uk[0], S.Uk[1], S.Uk[2], S.thl_m, 1.0, S.tend);
      oracle_diffuse(c, S.nu_s, 1.0 / c->Pr, S.thl_m, S.tmp);
      for (size_t q = 0; q < n; ++q) S.tend[q] += S.tmp[q];
      oracle_radiation(c, S.ql_m, S.cpmpi_m, S.tmp);
      for (size_t q = 0; q < n; ++q) S.tend[q] += S.tmp[q];
      scalar_sources(c, &P, S.thl_m, c->shf / c->cpd, S.tend);
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
          thl[q] = S.thl_h[q] + c->dt / P.rho0[k] * S.tend[q];
      /* q_t */
      oracle_advect(c, S.Uk[0], S.Uk[1], S.Uk[2], S.qt_m, 1.0, S.tend);
      oracle_diffuse(c, S.nu_s, 1.0 / c->Sc, S.qt_m, S.tmp);
      for (size_t q = 0; q < n; ++q) S.tend[q] += S.tmp[q];
      scalar_sources(c, &P, S.qt_m, c->lhf / c->Lv0, S.tend);
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
          qt[q] = S.qt_h[q] + c->dt / P.rho0[k] * S.tend[q];

      /* --- momentum predictor with U^{n+1/2} = (U^k + U^n)/2 */
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
          for (int a = 0; a < 3; ++a) {
            S.Uh[a][q] = 0.5 * (S.Uk[a][q] + S.Un[a][q]);
            S.uh[a][q] = S.Uh[a][q] / P.rho0[k];
          }
      oracle_sgs_nu(c, S.uh[0], S.uh[1], S.uh[2], S.b_h, S.nu_m);
      oracle_sgs_momentum(c, S.nu_m, S.uh[0], S.uh[1], S.uh[2], S.sg[0], S.sg[1], S.sg[2]);
      for (int a = 0; a < 3; ++a) {
        oracle_advect(c, S.Uh[0], S.Uh[1], S.Uh[2], S.uh[a], vpar(c, a), S.R[a]);
        for (size_t q = 0; q < n; ++q) S.R[a][q] += S.sg[a][q];
      }
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q) {
          double r0 = P.rho0[k];
          S.R[2][q] += r0 * S.b_h[q];                       /* buoyancy */
          S.R[0][q] += c->fcor * (S.Uh[1][q] - r0 * c->vg); /* -f k x rho0 (u - u_g) */
          S.R[1][q] -= c->fcor * (S.Uh[0][q] - r0 * c->ug);
          for (int a = 0; a < 3; ++a)                        /* sponge */
            S.R[a][q] -= P.beta[k] * (S.Uh[a][q] - r0 * ugv[a]);
          S.psi[q] = P.alpha0[k] * p[q];
        }
      for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
          for (int i = 0; i < c->nx; ++i) {
            size_t q = id3(c, i, j, k);
            for (int a = 0; a < 3; ++a) {
              const int *e = UNIT[a];
              double g = (at(c, S.psi, i + e[0], j + e[1], k + e[2], 1.0) -
                          at(c, S.psi, i - e[0], j - e[1], k - e[2], 1.0)) / (2.0 * spacing(c, a));
              S.Uhat[a][q] = S.Un[a][q] + c->dt * (-P.rho0[k] * g + S.R[a][q]);
            }
          }

      /* --- pressure correction */
      oracle_divergence(c, S.Uhat[0], S.Uhat[1], S.Uhat[2], S.rhs);
      oracle_app_a(c, S.phi_lag, S.tmp);
      for (int k = 0; k < c->nz; ++k)
        for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
          S.rhs[q] = P.alpha0[k] / c->dt * S.rhs[q] - S.tmp[q];
      double mr = fsum(c, S.rhs) / (double)n;
      for (size_t q = 0; q < n; ++q) S.rhs[q] -= mr;
      memset(S.phi, 0, n * sizeof(double));
      int guessed = 0;
      if (c->guess == 1 && it == 0) {
        for (int k = 0; k < c->nz; ++k)
          for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
            S.phi[q] = P.alpha0[k] * (p[q] - hist[q]);
        memcpy(hist, p, n * sizeof(double));
        guessed = 1;
      } else if (c->guess == 2 && step > 0) {
        memcpy(S.phi, hist + (size_t)it * n, n * sizeof(double));
        guessed = 1;
      }
      osolve st;
      int fixed = replay ? replay[solve] : 0;
      rc = poisson_solve(c, S.rhs, S.phi, fixed, guessed, zero_sweeps[it], &st);
      if (st.guess == 0 || st.guess == 2) zero_sweeps[it] = st.sweeps;
      else if (st.guess == 3) zero_sweeps[it] = st.sweeps - st.guess_sweeps;
      if (rec) rec[solve] = st;
      ++solve;
      if (rc) break;
      if (c->guess == 2) memcpy(hist + (size_t)it * n, S.phi, n * sizeof(double));

      /* --- projection: U^{k+1} = U_hat - dt rho0 grad_c phi, p += rho0 phi */
      for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
          for (int i = 0; i < c->nx; ++i) {
            size_t q = id3(c, i, j, k);
            for (int a = 0; a < 3; ++a) {
              const int *e = UNIT[a];
              double g = (at(c, S.phi, i + e[0], j + e[1], k + e[2], 1.0) -
                          at(c, S.phi, i - e[0], j - e[1], k - e[2], 1.0)) / (2.0 * spacing(c, a));
              S.Uk[a][q] = S.Uhat[a][q] - c->dt * P.rho0[k] * g;
            }
            p[q] += P.rho0[k] * S.phi[q];
          }
      memcpy(S.phi_lag, S.phi, n * sizeof(double));
    }
    for (int k = 0; k < c->nz; ++k)
      for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
        for (int a = 0; a < 3; ++a) vel[a][q] = S.Uk[a][q] / P.rho0[k];
  }

  if (dbg) {
    if (dbg->b_half) memcpy(dbg->b_half, S.b_h, n * sizeof(double));
    if (dbg->nu) memcpy(dbg->nu, S.nu_m, n * sizeof(double));
    if (dbg->rhs) memcpy(dbg->rhs, S.rhs, n * sizeof(double));
    if (dbg->phi) memcpy(dbg->phi, S.phi, n * sizeof(double));
    double *uh[3] = {dbg->uhat, dbg->vhat, dbg->what};
    for (int a = 0; a < 3; ++a)
      if (uh[a])
        for (int k = 0; k < c->nz; ++k)
          for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q)
            uh[a][q] = S.Uhat[a][q] / P.rho0[k];
  }
  free(hist);
  free(zero_sweeps);
  ostate_free(&S);
  prof_free(&P);
  return rc;
}

/* -------------------------------------------------------- diagnostics */

int oracle_diagnostics(const ocfg *c, const double *u, const double *v, const double *w,
                       const double *thl, const double *qt, double *scalars, double *profiles) {
  if (check_cfg(c)) return -1;
  size_t n = ncell(c);
  oprof P;
  if (prof_make(c, &P)) return -1;
  double *U = malloc(n * sizeof(double)), *V = malloc(n * sizeof(double));
  double *W = malloc(n * sizeof(double)), *D = malloc(n * sizeof(double));
  double *ql = malloc(n * sizeof(double)), *b = malloc(n * sizeof(double));
  if (!U || !V || !W || !D || !ql || !b) {
    free(U); free(V); free(W); free(D); free(ql); free(b); prof_free(&P);
    return -1;
  }
  oracle_thermo(c, thl, qt, NULL, ql, NULL, b);
  double dV = c->dx * c->dy * c->dz;
  double sth = 0, sqt = 0, ke = 0, cfl = 0;
  for (int k = 0; k < c->nz; ++k)
    for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q) {
      double r0 = P.rho0[k];
      U[q] = r0 * u[q]; V[q] = r0 * v[q]; W[q] = r0 * w[q];
      sth += r0 * thl[q] * dV;
      sqt += r0 * qt[q] * dV;
      ke += 0.5 * r0 * (u[q] * u[q] + v[q] * v[q] + w[q] * w[q]) * dV;
      double cf = fabs(u[q]) * c->dt / c->dx + fabs(v[q]) * c->dt / c->dy + fabs(w[q]) * c->dt / c->dz;
      if (cf > cfl) cfl = cf;
    }
  oracle_divergence(c, U, V, W, D);
  double dmax = 0;
  for (size_t q = 0; q < n; ++q) if (fabs(D[q]) > dmax) dmax = fabs(D[q]);
  if (scalars) {
    scalars[0] = sth; scalars[1] = sqt; scalars[2] = fnorm2(c, D); scalars[3] = dmax;
    scalars[4] = cfl; scalars[5] = ke;
  }
  if (profiles) {
    int nz = c->nz;
    double inv = 1.0 / ((double)c->nx * c->ny);
    for (int k = 0; k < nz; ++k) {
      double s[9] = {0};
      for (size_t q = (size_t)k * c->nx * c->ny; q < (size_t)(k + 1) * c->nx * c->ny; ++q) {
        s[0] += thl[q]; s[1] += qt[q]; s[2] += ql[q]; s[3] += u[q]; s[4] += v[q];
        s[5] += w[q]; s[6] += w[q] * w[q]; s[7] += w[q] * w[q] * w[q]; s[8] += b[q];
      }
      for (int a = 0; a < 9; ++a) profiles[a * nz + k] = s[a] * inv;
    }
  }
  free(U); free(V); free(W); free(D); free(ql); free(b);
  prof_free(&P);
  return 0;
}
