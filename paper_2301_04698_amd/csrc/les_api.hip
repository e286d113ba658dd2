// C ABI of the LES library (include/les.h): validation, workspace layout,
// reference state, and the stream-ordered orchestration of one time step
// of the paper's iterative predictor-corrector scheme (Sec. 2.4).
#include "les.h"
#include "les_cnn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "api_util.h"
#include "cnn_internal.h"
#include "les_internal.h"

using namespace lesmi;

namespace {

// Workspace fields (ids documented in les.h).
enum Field {
  F_UN = 0, F_VN, F_WN, F_THL_H, F_QT_H, F_THL_M, F_QT_M, F_UH, F_VH, F_WH,
  F_B_H, F_B_M, F_QL_M, F_CPMPI_M, F_NU_S, F_NU_M, F_RAD, F_RHS, F_PHI0, F_PHI1,
  F_PHI2, F_PHI3, F_PM2, F_GUESS, F_RHSD,
  F_COUNT
};

constexpr size_t kAlign = 256;
constexpr int kProfT = 7;  // storage-type profiles
constexpr int kTimeEvery = 4;  // time_sweeps: every 4th run of plain sweeps is timed
constexpr int kPartialCap = kPartials + 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
size_t mean_d_count(size_t nz) { return 5 * nz + 2; }
size_t pbar_index(size_t nz) { return 2 * nz; }

struct Layout {
  size_t field[F_COUNT];
  size_t prof_d;    // 4 x nz doubles: p0, lnp, alpha0, rho0
  size_t prof_t;    // 7 x nz elems: rho0, alpha0, beta, wsub, pgz, cbar, phigz
  size_t lvl_part;  // kPartials doubles: per-level partial sums
  size_t mean_d;    // kMeanD(nz) doubles: rsub, phibar, pbar (nz each), gbar, dbar (nz + 1
                    // each: level means and their mean), the FP64 mean-mode state
  size_t vert;      // LES_MEAN_EXACT: 5 nx ny + nx + ny doubles (column means of the
                    // rhs, of a guess and of a correction; the vertically uniform part;
                    // transform work; cas tables along x and y)
  size_t partials;  // kPartialCap doubles
  size_t partials2; // kPartials doubles: every other residual check's partials
  size_t ctl;       // SolveCtl
  size_t diag;      // nz x kDiagStride doubles
  size_t hist;      // n_subiter fields: previous step's solutions (history guess)
  // learned guess: residual (FP32), network input (bf16), two 16-channel
  // activations (bf16), parameters (FP32) and their bf16 copy, scales
  size_t cnn_r, cnn_a0, cnn_act[2], cnn_params, cnn_packed, cnn_sc;
  size_t total;
};

int validate(const les_config *c) {
  if (!c) return fail(LES_ERR_ARG, "config is NULL");
  if (c->nx < 2 || c->ny < 1 || c->nz < 4 || c->nz > 65535)
    return fail(LES_ERR_ARG, "grid %dx%dx%d: nx must be >= 2, ny >= 1 and 4 <= nz <= 65535",
                c->nx, c->ny, c->nz);
  // A z plane of one field stays within 2 GiB (the stencil kernels address
  // a plane with 32-bit byte offsets); at most 2^34 cells.
  const int64_t elem = c->precision == LES_FP64 ? 8 : 4;
  if ((int64_t)c->nx * c->ny * elem > (int64_t)1 << 31 ||
      (int64_t)c->nx * c->ny * c->nz > (int64_t)1 << 34)
    return fail(LES_ERR_ARG, "grid too large: at most 2 GiB per z plane and 2^34 cells");
  if (!(c->dx > 0) || !(c->dy > 0) || !(c->dz > 0) || !(c->dt > 0))
    return fail(LES_ERR_ARG, "dx, dy, dz, dt must be > 0");
  if (c->precision != LES_FP64 && c->precision != LES_FP32)
    return fail(LES_ERR_ARG, "precision must be LES_FP64 or LES_FP32");
  if (c->n_subiter < 1 || c->n_subiter > 64) return fail(LES_ERR_ARG, "n_subiter must be in [1, 64]");
  if (c->poisson_scheme != LES_JACOBI && c->poisson_scheme != LES_CHEBYSHEV)
    return fail(LES_ERR_ARG, "unknown poisson_scheme %d", c->poisson_scheme);
  if (c->poisson_check_every < 1) return fail(LES_ERR_ARG, "poisson_check_every must be >= 1");
  if (c->poisson_max_sweeps < 1 || c->poisson_max_sweeps > 1000000000)
    return fail(LES_ERR_ARG, "poisson_max_sweeps out of range");
  if (!(c->poisson_tol > 0)) return fail(LES_ERR_ARG, "poisson_tol must be > 0");
  if (!(c->jacobi_omega >= 0) || c->jacobi_omega >= 2)
    return fail(LES_ERR_ARG, "jacobi_omega must be in [0, 2)");
  if (c->satadj_maxit < 0 || c->satadj_maxit > 1000) return fail(LES_ERR_ARG, "satadj_maxit out of range");
  if (c->sweeps_per_launch < 0 || c->sweeps_per_launch > kMaxSweepsPerLaunch)
    return fail(LES_ERR_ARG, "sweeps_per_launch must be in [0, %d]", kMaxSweepsPerLaunch);
  if (!(c->p00 > 0) || !(c->theta0 > 0) || !(c->Rd > 0) || !(c->Rv > 0) || !(c->cpd > 0))
    return fail(LES_ERR_ARG, "thermodynamic constants must be > 0");
  const double top = c->nz * c->dz;
  if (!(1.0 - c->g * top / (c->cpd * c->theta0) > 0))
    return fail(LES_ERR_ARG, "domain top above the adiabatic atmosphere's height");
  if (c->sponge_frac < 0 || c->sponge_frac > 1) return fail(LES_ERR_ARG, "sponge_frac must be in [0, 1]");
  if (c->advection != LES_QUICK && c->advection != LES_WENO3)
    return fail(LES_ERR_ARG, "unknown advection scheme %d", c->advection);
  if (c->wall != LES_NO_SLIP && c->wall != LES_FREE_SLIP)
    return fail(LES_ERR_ARG, "unknown wall condition %d", c->wall);
  if (!(c->nu_const >= 0) || c->nu_const > 1e6)
    return fail(LES_ERR_ARG, "nu_const must be in [0, 1e6]");
  if (c->phase != LES_PHASE_HEAVISIDE && c->phase != LES_PHASE_RAMP)
    return fail(LES_ERR_ARG, "unknown phase partition %d", c->phase);
  if (c->phase == LES_PHASE_RAMP && !(c->T_ice > 0 && c->T_ice < c->Tf))
    return fail(LES_ERR_ARG, "T_ice must be in (0, Tf) for LES_PHASE_RAMP");
  if (c->guess < LES_GUESS_ZERO || c->guess > LES_GUESS_LEARNED3)
    return fail(LES_ERR_ARG, "unknown guess mode %d", c->guess);
  // the guess network addresses a z plane of 16-channel activations with
  // 32-bit element offsets
  if ((c->guess == LES_GUESS_LEARNED || c->guess == LES_GUESS_LEARNED3) &&
      (int64_t)c->nx * c->ny * 16 >= (int64_t)1 << 31)
    return fail(LES_ERR_ARG, "learned guess: at most 2^27 cells per z plane");
  if (c->mean_mode != LES_MEAN_SWEPT && c->mean_mode != LES_MEAN_LEVEL &&
      c->mean_mode != LES_MEAN_EXACT)
    return fail(LES_ERR_ARG, "unknown mean mode %d", c->mean_mode);
  if (c->guess_passes < 0 || c->guess_passes > 4 ||
      (c->guess_passes > 1 && c->guess != LES_GUESS_LEARNED))
    return fail(LES_ERR_ARG, "guess_passes must be in [0, 4], above 1 only with LES_GUESS_LEARNED");
  return LES_OK;
}

size_t elem_size(const les_config *c) { return c->precision == LES_FP64 ? 8 : 4; }

// Guess modes that keep each sub-iteration's previous solution; that keep
// the previous step's pressure; the input channels of the guess network (0:
// none).
bool uses_hist(const les_config *c) {
  return c->guess == LES_GUESS_PREVIOUS || c->guess == LES_GUESS_LEARNED;
}
bool uses_pm2(const les_config *c) {
  return c->guess == LES_GUESS_EXTRAPOLATE || c->guess == LES_GUESS_LEARNED3;
}
int cnn_inputs_of(const les_config *c) {
  return c->guess == LES_GUESS_LEARNED ? 1 : c->guess == LES_GUESS_LEARNED3 ? 3 : 0;
}

Layout layout_of(const les_config *c) {
  Layout L;
  const size_t n = (size_t)c->nx * c->ny * c->nz;
  const size_t es = elem_size(c);
  size_t off = 0;
  for (int f = 0; f < F_COUNT; ++f) {
    L.field[f] = off;
    off = align_up(off + n * es);
  }
  L.prof_d = off;
  off = align_up(off + 4 * (size_t)c->nz * sizeof(double));
  L.prof_t = off;
  off = align_up(off + kProfT * (size_t)c->nz * es);
  L.lvl_part = off;
  off = align_up(off + kPartials * sizeof(double));
  L.mean_d = off;
  off = align_up(off + mean_d_count(c->nz) * sizeof(double));
  L.vert = off;
  if (c->mean_mode == LES_MEAN_EXACT)
    off = align_up(off + (5 * (size_t)c->nx * c->ny + c->nx + c->ny) * sizeof(double));
  L.partials = off;
  off = align_up(off + kPartialCap * sizeof(double));
  L.partials2 = off;
  off = align_up(off + kPartials * sizeof(double));
  L.ctl = off;
  off = align_up(off + sizeof(SolveCtl));
  L.diag = off;
  off = align_up(off + (size_t)c->nz * kDiagStride * sizeof(double));
  L.hist = off;  // LES_GUESS_LEARNED3: one field, the extrapolated base
  if (uses_hist(c)) off = align_up(off + (size_t)c->n_subiter * n * es);
  else if (c->guess == LES_GUESS_LEARNED3) off = align_up(off + n * es);
  const int ci = cnn_inputs_of(c);
  const bool cnn = ci > 0;
  L.cnn_r = off;
  if (cnn) off = align_up(off + n * sizeof(float));
  L.cnn_a0 = off;
  if (cnn) off = align_up(off + n * ci * sizeof(uint16_t));
  for (int q = 0; q < 2; ++q) {
    L.cnn_act[q] = off;
    if (cnn) off = align_up(off + n * kCnnCh * sizeof(uint16_t));
  }
  L.cnn_params = off;
  if (cnn) off = align_up(off + (size_t)cnn_param_count(ci) * sizeof(float));
  L.cnn_packed = off;
  if (cnn) off = align_up(off + (size_t)cnn_param_count(ci) * sizeof(uint16_t));
  L.cnn_sc = off;
  if (cnn) off = align_up(off + 4 * sizeof(double));
  L.total = off;
  return L;
}

}  // namespace

struct les_handle {
  les_config cfg;
  les_buffers buf;
  hipStream_t stream;
  Layout lay;
  Grid grid;
  Thermo thermo;
  double mu_min, mu_max;
  int sweeps_per_launch;  // temporal blocking depth of the Poisson sweeps
  SolveCtl *ctl_host;  // pinned mirror for the final read-back
  int64_t *poll_word;      // pinned, coherent: (decision number << 32) | done, written
                           // by the kernel deciding each residual test
  int64_t *poll_word_dev;  // device view of poll_word
  double *diag_host;   // pinned, nz x kDiagStride
  hipEvent_t ev_a, ev_b, ev_s0, ev_s1;
  std::vector<hipEvent_t> ev_sweep;  // pool bracketing runs of plain sweeps
  bool broken;
  std::vector<char> hist_valid;  // per sub-iteration: history holds a solution
  std::vector<int32_t> zero_sweeps;  // per sub-iteration: sweeps of its last pass from the
                                     // zero start (a kept guess's budget; 0 none yet)
  bool cnn_bound;                // learned guess: parameters bound
  float cnn_alpha;               // its leaky ReLU slope
  int64_t steps_done;            // time steps taken since les_init (or the imported count)
};

namespace {

char *ws(const les_handle *h, size_t off) { return (char *)h->buf.workspace + off; }

// Extreme nonzero eigenvalues of -D^{-1} L (compact Laplacian, periodic x/y,
// mirror-Neumann z) on the modes the sweeps act on: sums of
// (2 - 2 cos theta)/Delta^2 per axis over D.  With LES_MEAN_EXACT those
// modes have both horizontal and vertical structure, so the smallest is
// the smallest horizontal eigenvalue plus the smallest vertical one.
void jacobi_spectrum(const les_config *c, double *lo, double *hi) {
  const double pi = 3.14159265358979323846;
  const double ax = 1.0 / (c->dx * c->dx), ay = 1.0 / (c->dy * c->dy), az = 1.0 / (c->dz * c->dz);
  const double D = 2.0 * (ax + ay + az);
  auto per = [&](int n, int m) { return 2.0 - 2.0 * std::cos(2.0 * pi * m / n); };
  auto mir = [&](int n, int m) { return 2.0 - 2.0 * std::cos(pi * m / n); };
  // a periodic axis of one cell has only its constant mode
  double h = per(c->nx, 1) * ax;  // nx >= 2
  if (c->ny > 1) h = std::min(h, per(c->ny, 1) * ay);
  const double z1 = mir(c->nz, 1) * az;
  *lo = (c->mean_mode == LES_MEAN_EXACT ? h + z1 : std::min(h, z1)) / D;
  *hi = (per(c->nx, c->nx / 2) * ax + per(c->ny, c->ny / 2) * ay + mir(c->nz, c->nz - 1) * az) / D;
}

template <typename T>
struct View {
  T *f[F_COUNT];
  Profiles<T> P;
  Dyn<T> dyn;
  double *partials, *partials2;
  SolveCtl *ctl;
  double *diag;
  T *u, *v, *w, *thl, *qt, *p;
  // mean-mode state: level partials, per-level centring values, the
  // horizontally uniform part of the current solution, of a guess, of p' and
  // of a correction (gbar, dbar: nz level means and their mean)
  double *lvl_part, *rsub, *phibar, *gbar, *pbar, *dbar;
  // vertically uniform part (LES_MEAN_EXACT): column means of the rhs
  // (cmean), of a guess (gv), of a correction (dv); the part itself (pv);
  // transform work; cas tables
  double *cmean, *gv, *dv, *pv, *work, *tab_x, *tab_y;
  T *pgz_w, *cbar_w, *phigz_w;  // writable views of the profile terms
  int exact;                    // the horizontally uniform part solved exactly
  int vert;                     // the vertically uniform part too (LES_MEAN_EXACT)
};

template <typename T>
View<T> view_of(const les_handle *h) {
  View<T> V;
  for (int f = 0; f < F_COUNT; ++f) V.f[f] = (T *)ws(h, h->lay.field[f]);
  const int nz = h->cfg.nz;
  double *pd = (double *)ws(h, h->lay.prof_d);
  T *pt = (T *)ws(h, h->lay.prof_t);
  V.P.p0 = pd;
  V.P.lnp = pd + nz;
  V.P.alpha0 = pd + 2 * nz;
  V.P.rho0 = pd + 3 * nz;
  V.P.rho0_t = pt;
  V.P.alpha0_t = pt + nz;
  V.P.beta_t = pt + 2 * nz;
  V.P.wsub_t = pt + 3 * nz;
  V.P.pgz_t = V.pgz_w = pt + 4 * nz;
  V.P.cbar_t = V.cbar_w = pt + 5 * nz;
  V.P.phigz_t = V.phigz_w = pt + 6 * nz;
  V.lvl_part = (double *)ws(h, h->lay.lvl_part);
  double *md = (double *)ws(h, h->lay.mean_d);
  V.rsub = md;
  V.phibar = md + nz;
  V.pbar = md + pbar_index(nz);
  V.gbar = md + 3 * nz;
  V.dbar = md + 4 * nz + 1;
  V.exact = h->cfg.mean_mode != LES_MEAN_SWEPT;
  V.vert = h->cfg.mean_mode == LES_MEAN_EXACT;
  const size_t nxy = (size_t)h->cfg.nx * h->cfg.ny;
  double *vd = (double *)ws(h, h->lay.vert);
  V.cmean = vd;
  V.gv = vd + nxy;
  V.dv = vd + 2 * nxy;
  V.pv = vd + 3 * nxy;
  V.work = vd + 4 * nxy;
  V.tab_x = vd + 5 * nxy;
  V.tab_y = V.tab_x + h->cfg.nx;
  V.partials = (double *)ws(h, h->lay.partials);
  V.partials2 = (double *)ws(h, h->lay.partials2);
  V.ctl = (SolveCtl *)ws(h, h->lay.ctl);
  V.diag = (double *)ws(h, h->lay.diag);
  const les_config &c = h->cfg;
  Dyn<T> &d = V.dyn;
  d.dt = (T)c.dt;
  d.inv_dx = (T)(1.0 / c.dx);
  d.inv_dy = (T)(1.0 / c.dy);
  d.inv_dz = (T)(1.0 / c.dz);
  d.inv_2dx = (T)(0.5 / c.dx);
  d.inv_2dy = (T)(0.5 / c.dy);
  d.inv_2dz = (T)(0.5 / c.dz);
  d.fcor = (T)c.fcor;
  d.ug = (T)c.ug;
  d.vg = (T)c.vg;
  d.inv_pr = (T)(1.0 / c.Pr);
  d.inv_sc = (T)(1.0 / c.Sc);
  d.sfc_thl = (T)(c.shf / c.cpd);
  d.sfc_qt = (T)(c.lhf / c.Lv0);
  const double delta = std::cbrt(c.dx * c.dy * c.dz);
  d.smag_l2 = (T)((c.cs * delta) * (c.cs * delta));
  d.pr = (T)c.Pr;
  d.advection = c.advection;
  d.uv_par = c.wall == LES_FREE_SLIP ? T(1) : T(-1);
  d.nu_const = (T)c.nu_const;
  V.u = (T *)h->buf.u;
  V.v = (T *)h->buf.v;
  V.w = (T *)h->buf.w;
  V.thl = (T *)h->buf.thl;
  V.qt = (T *)h->buf.qt;
  V.p = (T *)h->buf.p;
  return V;
}

// Reference state (Sec. 2.1) on the host in FP64, uploaded into the
// workspace (FP64 copies for thermodynamics and reductions, storage-type
// copies for the stencils).  Returns after the upload completed.
template <typename T>
int upload_profiles(les_handle *h) {
  const les_config &c = h->cfg;
  const int nz = c.nz;
  std::vector<double> pd(4 * (size_t)nz);
  std::vector<T> pt(kProfT * (size_t)nz, T(0));
  const std::vector<double> md(mean_d_count(nz), 0.0);  // no mean-mode part yet
  const double H = nz * c.dz, zs = (1.0 - c.sponge_frac) * H;
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < nz; ++k) {
    const double z = (k + 0.5) * c.dz;
    const double base = 1.0 - c.g * z / (c.cpd * c.theta0);
    const double p0 = c.p00 * std::pow(base, c.cpd / c.Rd);   // hydrostatic, adiabatic
    const double T0 = c.theta0 * std::pow(p0 / c.p00, c.Rd / c.cpd);
    const double alpha0 = c.Rd * T0 / p0;                       // = 1 / rho0
    const double rho0 = p0 / (c.Rd * T0);
    double beta = 0.0;
    if (z >= zs && H > zs) {
      const double s = std::sin(0.5 * pi * (z - zs) / (H - zs));
      beta = c.sponge_max * s * s;
    }
    pd[k] = p0;
    pd[nz + k] = std::log(p0 / c.p00);
    pd[2 * nz + k] = alpha0;
    pd[3 * nz + k] = rho0;
    pt[k] = (T)rho0;
    pt[nz + k] = (T)alpha0;
    pt[2 * nz + k] = (T)beta;
    pt[3 * nz + k] = (T)(c.wsub_div * z);
  }
  HIP_TRY(hipMemcpyAsync(ws(h, h->lay.prof_d), pd.data(), pd.size() * sizeof(double),
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(ws(h, h->lay.prof_t), pt.data(), pt.size() * sizeof(T),
                         hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(ws(h, h->lay.mean_d), md.data(), md.size() * sizeof(double),
                         hipMemcpyHostToDevice, h->stream));
  // cas(2 pi m / n) = cos + sin, m < n, for the transforms of the
  // vertically uniform part
  std::vector<double> tab;
  if (c.mean_mode == LES_MEAN_EXACT) {
    for (int n : {c.nx, c.ny})
      for (int m = 0; m < n; ++m) {
        const double t = 2.0 * pi * m / n;
        tab.push_back(std::cos(t) + std::sin(t));
      }
    const size_t nxy = (size_t)c.nx * c.ny;
    HIP_TRY(hipMemcpyAsync((double *)ws(h, h->lay.vert) + 5 * nxy, tab.data(),
                           tab.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LES_OK;
}

// Device time of the runs of consecutive plain (non-check) sweeps of one
// solve that lie before the returned iterate.
struct SweepTiming {
  bool enabled = false;
  double seconds = 0.0;
  int64_t sweeps = 0;
};

// Centred right-hand side of a solve into F_RHS (rhs_in may be F_RHS
// itself): the mean removed and, with the horizontally uniform part solved
// exactly, the horizontal mean of every level, whose part of the solution
// goes to V.phibar (zero otherwise).  With the vertically uniform part
// solved exactly too (V.vert), that part V.pv from the column means of the
// right-hand side, and the sweeps' right-hand side F_RHSD = F_RHS without
// them (Sec. 2.3 with the uniform modes split off; Eq. 7's operator).
// Resets the control block; the stopping test is relative to
// ||rhs_in - mean||, the norm of the whole centred right-hand side.
template <typename T>
int prepare_rhs(les_handle *h, View<T> &V, const T *rhs_in, int max_sweeps, bool fixed) {
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  const double tol = h->cfg.poisson_tol;
  launch_ctl_reset(V.ctl, max_sweeps, fixed ? 1 : 0, s);
  launch_level_sum<T>(g, rhs_in, V.lvl_part, s);
  launch_mean_mode(g, V.lvl_part, V.exact, V.ctl, V.rsub, V.phibar, s);
  if (V.vert) {
    launch_column_mean<T>(g, rhs_in, V.cmean, s);
    launch_vertical_solve(g, V.cmean, V.ctl, V.tab_x, V.tab_y, V.work, V.pv, s);
  }
  // the sweeps start from zero in F_PHI0
  launch_rhs_center<T>(g, rhs_in, V.f[F_RHS], V.f[F_PHI0], V.rsub, V.ctl, V.partials, s);
  launch_final(V.partials, level_parts(g) * g.nz, kFinalRhsNorm, V.ctl, (double)g.n, tol * tol,
               0, nullptr, s);
  if (V.vert) launch_remove_columns<T>(g, V.f[F_RHS], V.cmean, V.ctl, V.f[F_RHSD], s);
  LAUNCH_TRY();
  return LES_OK;
}

// The right-hand side the sweeps take from the zero start.
template <typename T>
T *sweep_rhs(View<T> &V) {
  return V.vert ? V.f[F_RHSD] : V.f[F_RHS];
}

// Starting iterate `guess` of the solve prepared by prepare_rhs, in defect
// form: F_RHSD = (zero start's rhs) - L(guess - gbar - gv), gbar its
// horizontal means per level when those are solved exactly (already part
// of V.phibar), gv its column means when those are (already part of V.pv).
// The guess is kept if always_keep or its residual is below the zero
// start's; a dropped guess leaves F_RHSD the zero start's right-hand side.
template <typename T>
int prepare_guess(les_handle *h, View<T> &V, const T *guess, bool always_keep) {
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  launch_level_sum<T>(g, guess, V.lvl_part, s);
  launch_level_mean(g, V.lvl_part, V.exact, V.gbar, s);
  if (V.vert) launch_column_mean<T>(g, guess, V.gv, s);
  launch_guess_gate<T>(g, sweep_rhs(V), guess, V.exact ? V.gbar : nullptr,
                       V.vert ? V.gv : nullptr, V.f[F_RHSD], V.partials, V.ctl,
                       always_keep ? 1 : 0, s);
  LAUNCH_TRY();
  return LES_OK;
}

// Sweeps on L phi = rhs from zero until the device-side residual test
// (relative to the reference norm in the control block) stops them, the cap
// (`cap` if > 0, which the control block must hold too, else the
// configuration's) or exactly `fixed` sweeps.  *result: the buffer holding the returned
// iterate; *out: the control block as it ended (the stream is synchronized).
template <typename T>
int run_sweeps(les_handle *h, View<T> &V, const T *rhs, int fixed, int cap, SolveCtl *out,
               T **result, SweepTiming *timing) {
  const les_config &c = h->cfg;
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  const int max_sweeps = fixed > 0 ? fixed : (cap > 0 ? cap : c.poisson_max_sweeps);
  const int every = c.poisson_check_every;
  const bool cheb = c.poisson_scheme == LES_CHEBYSHEV;
  const double gamma = 2.0 / (h->mu_min + h->mu_max);
  const double rho = (h->mu_max - h->mu_min) / (h->mu_max + h->mu_min);
  const double omega_j = cheb ? gamma : (c.jacobi_omega > 0 ? c.jacobi_omega : gamma);
  const int smax = h->sweeps_per_launch;

  // Launches of up to smax sweeps, made one at a time; a residual check at
  // sweep m is computed by the launch that starts at m (its input iterate
  // is phi_m), so launches are cut at check positions.  Checks at every
  // `every`-th sweep and at the cap (or only at the fixed count).
  auto is_check = [&](int mm) {
    return fixed > 0 ? (mm == max_sweeps) : (mm % every == 0 || mm == max_sweeps);
  };
  struct Launch {
    int m, S;
    bool check;
  };
  auto launch_at = [&](int mm) {
    Launch L{mm, 1, is_check(mm)};
    if (mm < max_sweeps)
      while (L.S < smax && mm + L.S < max_sweeps && !is_check(mm + L.S)) ++L.S;
    return L;
  };

  // Four iterate buffers: a launch reads (prev, cur) and writes its last two
  // iterates into the two buffers it does not read.  The last few checks
  // remember the buffer of their input iterate; the decisive one is among
  // them (the host stops queueing `lag` checks after the device decided).
  T *buf[4] = {V.f[F_PHI0], V.f[F_PHI1], V.f[F_PHI2], V.f[F_PHI3]};
  int cur = 0, prev = -1;
  constexpr int kRecent = 16;
  int recent_m[kRecent], recent_buf[kRecent], nrecent = 0;

  // Queue launches; the device stops applying them once a check succeeds.
  // The kernel deciding test number c writes (c << 32) | done into a pinned,
  // coherent host word; before queueing past test c the host waits for the
  // word of test c - lag (so it stays a bounded number of tests ahead) and
  // stops once a decided test says done.  No event or copy per test: each
  // of those cost the stream several microseconds.
  const int lag = 2;
  size_t npending = 0;
  struct Run {
    int first, last;
  };
  constexpr size_t kMaxRuns = 4096;  // timed runs per solve (a sample)
  std::vector<Run> runs;
  const bool timed = timing && timing->enabled;
  int run_first = -1, run_seen = 0;
  bool prev_plain = false;  // the previous launch was a full plain one
  double wc_prev = 1.0;  // Chebyshev weight recurrence
  // pending residual check (decided by the next launch) and the host poll:
  // a copy of the control block after each decision, read `lag` checks later
  int pend_m = -1, pend_np = 0, nchecks = 0;
  const double *pend_parts = nullptr;
  volatile int64_t *word = h->poll_word;
  *word = 0;  // the previous solve's launches are complete (it ended synchronized)
  // the number the next decision writes
  auto next_seq = [&]() { return (int)npending + 1; };
  auto poll = [&](bool &done) -> hipError_t {
    ++npending;  // decision npending is queued
    if (npending <= (size_t)lag) return hipSuccess;
    const int64_t want = (int64_t)(npending - lag);
    for (uint64_t it = 1;; ++it) {
      const int64_t v = *word;
      if ((v >> 32) >= want || (v & 0xffffffff) != 0) {
        done = (v & 0xffffffff) != 0;
        return hipSuccess;
      }
      if (it % 256 == 0) {  // an idle stream has run every queued launch
        const hipError_t q = hipStreamQuery(s);
        if (q != hipErrorNotReady) {
          if (q != hipSuccess) return q;
          const int64_t v2 = *word;
          done = (v2 & 0xffffffff) != 0;
          return hipSuccess;
        }
      }
      std::this_thread::yield();
    }
  };
  Launch L = launch_at(0);
  int last_m = 0;
  for (bool more = true; more;) {
    const Launch nextL = L.m + L.S <= max_sweeps ? launch_at(L.m + L.S) : Launch{-1, 0, false};
    const bool has_next = nextL.m >= 0;
    last_m = L.m;
    const bool plain_full = !L.check && L.S == smax;
    // a run starts at a plain launch after a check; every kTimeEvery-th run
    // is bracketed by events (each event costs the stream a few us)
    const bool run_start = plain_full && !prev_plain;
    if (run_start) ++run_seen;
    if (timed && run_start && run_first < 0 && (run_seen - 1) % kTimeEvery == 0 &&
        runs.size() < kMaxRuns) {
      const size_t e = 2 * runs.size();
      while (h->ev_sweep.size() < e + 2) {
        hipEvent_t ev;
        HIP_TRY(hipEventCreate(&ev));
        h->ev_sweep.push_back(ev);
      }
      HIP_TRY(hipEventRecord(h->ev_sweep[e], s));
      run_first = L.m;
    }
    double wc[4] = {1.0, 1.0, 1.0, 1.0};
    for (int q = 0; q < L.S; ++q) {  // weight of sweep L.m + q
      const int mm = L.m + q;
      double w = 1.0;
      if (cheb) {
        if (mm == 0) w = 1.0;
        else if (mm == 1) w = 1.0 / (1.0 - 0.5 * rho * rho);
        else w = 1.0 / (1.0 - 0.25 * rho * rho * wc_prev);
      }
      wc[q] = w;
      wc_prev = w;
    }
    int free_[4], nf = 0;
    for (int q = 0; q < 4; ++q)
      if (q != cur && q != prev) free_[nf++] = q;
    const int out_last = L.S == 1 ? free_[0] : free_[1];
    const int out_prev = L.S == 1 ? -1 : free_[0];
    if (L.check) {
      recent_m[nrecent % kRecent] = L.m;
      recent_buf[nrecent % kRecent] = cur;
      ++nrecent;
    }
    // A check left pending by the previous launch is decided by this one
    // (block 0 reduces its partials); checks alternate partial buffers so a
    // checking launch can decide the check before it.
    const bool decides = pend_m >= 0 && L.S == 1;
    double *parts = (nchecks & 1) ? V.partials2 : V.partials;
    // The first Chebyshev sweep has weight 1: the plain weighted-Jacobi
    // sweep, which must not read the (uninitialised) previous iterate.
    launch_tsweep<T>(g, L.S, cheb, L.check, L.m == 0, omega_j, wc, buf[cur],
                     prev >= 0 ? buf[prev] : nullptr, buf[out_last],
                     out_prev >= 0 ? buf[out_prev] : nullptr, rhs, V.ctl, parts,
                     decides ? pend_parts : nullptr, decides ? pend_np : 0, decides ? pend_m : -1,
                     decides ? h->poll_word_dev : nullptr, next_seq(), s);
    if (L.S == 1) {
      prev = cur;
    } else {
      prev = out_prev;
    }
    cur = out_last;
    const bool next_plain_full = has_next && !nextL.check && nextL.S == smax;
    if (timed && run_first >= 0 && !next_plain_full) {
      HIP_TRY(hipEventRecord(h->ev_sweep[2 * runs.size() + 1], s));
      runs.push_back(Run{run_first, L.m + L.S - 1});
      run_first = -1;
    }
    bool stop = false;
    if (decides) {
      pend_m = -1;
      LAUNCH_TRY();
      HIP_TRY(poll(stop));
    }
    if (L.check) {
      ++nchecks;
      // partial sums come from this launch's own block decomposition; the
      // next launch decides unless it is a two-sweep launch or there is none
      const int np = tsweep_blocks(g, L.S, sizeof(T) == 8);
      if (L.S == 1 && has_next && nextL.S == 1) {
        pend_m = L.m;
        pend_parts = parts;
        pend_np = np;
      } else {
        launch_final_check(parts, np, V.ctl, (double)g.n, L.m, h->poll_word_dev, next_seq(), s);
        LAUNCH_TRY();
        bool stop2 = false;
        HIP_TRY(poll(stop2));
        stop = stop || stop2;
      }
    }
    prev_plain = plain_full;
    more = !stop && has_next;
    if (more) L = nextL;
  }
  if (pend_m >= 0) {  // a check no later launch decided (the loop stopped early)
    launch_final_check(pend_parts, pend_np, V.ctl, (double)g.n, pend_m, nullptr, 0, s);
    LAUNCH_TRY();
  }
  LAUNCH_TRY();
  if (timed && run_first >= 0) {  // loop left inside a run
    HIP_TRY(hipEventRecord(h->ev_sweep[2 * runs.size() + 1], s));
    runs.push_back(Run{run_first, last_m});
  }
  HIP_TRY(hipMemcpyAsync(&h->ctl_host[0], V.ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const SolveCtl &r = h->ctl_host[0];
  *out = r;
  if (timed) {
    // only runs made entirely of sweeps applied before the returned iterate
    for (size_t q = 0; q < runs.size(); ++q) {
      if (runs[q].last >= r.stop_m) continue;
      float rms = 0.f;
      HIP_TRY(hipEventElapsedTime(&rms, h->ev_sweep[2 * q], h->ev_sweep[2 * q + 1]));
      timing->seconds += rms * 1e-3;
      timing->sweeps += runs[q].last - runs[q].first + 1;
    }
  }
  if (r.done == 0 || r.stop_m < 0)
    return fail(LES_ERR_STATE, "Poisson solve ended without a decision");
  int res_buf = -1;
  for (int q = 0; q < kRecent && q < nrecent; ++q)
    if (recent_m[q] == r.stop_m) res_buf = recent_buf[q];
  if (res_buf < 0) return fail(LES_ERR_STATE, "Poisson solve stopped at an unchecked sweep");
  *result = buf[res_buf];
  if (r.done == 2) return fail(LES_ERR_NONFINITE, "non-finite Poisson residual");
  return LES_OK;
}

// A whole solve after prepare_rhs (and prepare_guess if `guess`): the
// sweeps, then for a kept guess phi = guess - gbar + correction (with
// V.vert: the correction without its level and column means, plus pv, plus
// the guess without its level and column means) and the FP64 residual of
// that returned iterate.  gated: a kept guess whose solve
// reaches the cap, or (budget > 0) the first residual check at or beyond
// `budget` sweeps, or whose returned iterate misses the tolerance, is
// dropped and the sweeps repeated from the zero start (unless the sweep
// count is fixed).  The caller recorded h->ev_s0 before preparing the
// solve; st covers everything since.
template <typename T>
int solve_prepared(les_handle *h, View<T> &V, const T *guess, bool gated, int fixed, int budget,
                   les_solve_stats *st, T **result, SweepTiming *timing) {
  const Grid &g = h->grid;
  const les_config &c = h->cfg;
  hipStream_t s = h->stream;
  SolveCtl r;
  T *phi = nullptr;
  int cap = 0;
  if (guess && gated && fixed == 0 && budget > 0) {
    // a kept guess gets the budget (the gate's decision is read back first,
    // so a dropped guess's zero start keeps the whole cap)
    HIP_TRY(hipMemcpyAsync(&h->ctl_host[0], V.ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int every = c.poisson_check_every;
    const int64_t b = ((int64_t)budget + every - 1) / every * every;
    if (h->ctl_host[0].guess_kept && b < c.poisson_max_sweeps) {
      cap = (int)b;
      launch_ctl_limit(V.ctl, cap, s);
      LAUNCH_TRY();
    }
  }
  // With the vertically uniform part exact, every returned iterate is
  // assembled (the correction projected, plus pv and the guess) and its
  // residual taken against F_RHS.
  auto assemble = [&](T *x, const T *gs) -> int {
    launch_level_sum<T>(g, x, V.lvl_part, s);
    launch_level_mean(g, V.lvl_part, 1, V.dbar, s);
    launch_column_mean<T>(g, x, V.dv, s);
    launch_combine<T>(g, x, V.dbar, V.dv, V.pv, gs, V.gbar, V.gv, V.ctl, s);
    launch_returned_residual<T>(g, V.f[F_RHS], x, V.partials, V.ctl, s);
    LAUNCH_TRY();
    HIP_TRY(hipMemcpyAsync(&h->ctl_host[0], V.ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LES_OK;
  };
  int rc = run_sweeps<T>(h, V, guess ? V.f[F_RHSD] : sweep_rhs(V), fixed, cap, &r, &phi, timing);
  if (rc) return rc;
  int sweeps = r.stop_m, first = 0;
  int flag = guess ? (r.guess_kept ? 1 : 2) : 0;
  double res2 = r.res_norm2;
  // the returned iterate from the sweeps' phi and guess gs: its FP64
  // residual into res2 (r the control block as it ended)
  auto finish = [&](const T *gs) -> int {
    if (V.vert) {
      if ((rc = assemble(phi, gs))) return rc;
    } else {
      launch_add_guess<T>(g, gs, V.exact ? V.gbar : nullptr, V.ctl, phi, s);
      launch_returned_residual<T>(g, V.f[F_RHS], phi, V.partials, V.ctl, s);
      LAUNCH_TRY();
      HIP_TRY(hipMemcpyAsync(&h->ctl_host[0], V.ctl, sizeof(SolveCtl), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    r = h->ctl_host[0];
    res2 = r.res_out2;
    return LES_OK;
  };
  if (V.vert || (guess && r.guess_kept)) {
    if ((rc = finish(guess))) return rc;
    bool missed = r.done == 3 || !(res2 <= r.tol2);
    if (guess && r.guess_kept && gated && fixed == 0 && missed && r.done == 1) {
      // The sweeps met the test but the returned iterate (guess plus
      // correction and the exactly solved parts, rounded to the storage
      // precision) misses it: a near miss, not a bad guess.  Continue once
      // from that iterate as the guess (in F_GUESS) under the same cap, or
      // with no budget under the first pass's count (a continuation that
      // needs more than that is no near miss).
      int ccap = cap;
      if (ccap == 0) {
        const int every = c.poisson_check_every;
        const int64_t b = ((int64_t)std::max(sweeps, 1) + every - 1) / every * every;
        ccap = (int)std::min<int64_t>(b, c.poisson_max_sweeps);
      }
      HIP_TRY(hipMemcpyAsync(V.f[F_GUESS], phi, (size_t)g.n * sizeof(T), hipMemcpyDeviceToDevice,
                             s));
      launch_ctl_restart(V.ctl, c.poisson_max_sweeps, s);
      launch_zero<T>(g, V.f[F_PHI0], s);
      if (V.vert) launch_remove_columns<T>(g, V.f[F_RHS], V.cmean, V.ctl, V.f[F_RHSD], s);
      LAUNCH_TRY();
      if ((rc = prepare_guess<T>(h, V, V.f[F_GUESS], true))) return rc;
      launch_ctl_limit(V.ctl, ccap, s);
      LAUNCH_TRY();
      rc = run_sweeps<T>(h, V, V.f[F_RHSD], 0, ccap, &r, &phi, timing);
      if (rc) return rc;
      first = sweeps;
      sweeps += r.stop_m;
      flag = 4;
      if ((rc = finish(V.f[F_GUESS]))) return rc;
      missed = r.done == 3 || !(res2 <= r.tol2);
    }
    if (guess && r.guess_kept && gated && fixed == 0 && missed) {
      launch_ctl_restart(V.ctl, c.poisson_max_sweeps, s);
      launch_zero<T>(g, V.f[F_PHI0], s);
      // the zero start's right-hand side again (the defect overwrote it)
      if (V.vert) launch_remove_columns<T>(g, V.f[F_RHS], V.cmean, V.ctl, V.f[F_RHSD], s);
      LAUNCH_TRY();
      rc = run_sweeps<T>(h, V, sweep_rhs(V), 0, 0, &r, &phi, timing);
      if (rc) return rc;
      first = sweeps;
      sweeps += r.stop_m;
      res2 = r.res_norm2;
      flag = 3;
      if (V.vert) {  // guess_kept is 0 now: pv and the projected correction
        if ((rc = assemble(phi, guess))) return rc;
        r = h->ctl_host[0];
        res2 = r.res_out2;
        if (r.done == 1 && !(res2 <= r.tol2)) r.done = 3;
      }
    } else if (r.done == 1 && !(res2 <= r.tol2)) {
      r.done = 3;  // the returned iterate misses the tolerance
    }
  }
  HIP_TRY(hipEventRecord(h->ev_s1, s));
  HIP_TRY(hipEventSynchronize(h->ev_s1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, h->ev_s0, h->ev_s1));
  st->sweeps = sweeps;
  st->status = r.done == 1 ? 0 : 1;
  st->rhs_norm = std::sqrt(r.rhs_norm2);
  st->res_norm = std::sqrt(res2);
  st->seconds = ms * 1e-3;
  st->guess = flag;
  st->guess_sweeps = first;
  *result = phi;
  return LES_OK;
}

// Learned initial guess into the first iterate buffer.
template <typename T>
int cnn_guess(les_handle *h, View<T> &V, const T *rhs, const T *base, T *guess);

template <typename T>
int step_impl(les_handle *h, int32_t nsteps, const les_step_opts *opts, les_step_stats *stats) {
  View<T> V = view_of<T>(h);
  const les_config &c = h->cfg;
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  const size_t bytes = (size_t)g.n * sizeof(T);
  const int K = c.n_subiter;
  les_step_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  int rc_final = LES_OK;

  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, s));
  for (int step = 0; step < nsteps; ++step) {
    // step-start copies U^n, Phi^{n+1/2}
    HIP_TRY(hipMemcpyAsync(V.f[F_UN], V.u, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(V.f[F_VN], V.v, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(V.f[F_WN], V.w, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(V.f[F_THL_H], V.thl, bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(V.f[F_QT_H], V.qt, bytes, hipMemcpyDeviceToDevice, s));
    // b^{n+1/2}; at k = 0 the midpoint state equals Phi^{n+1/2}
    launch_thermo<T>(g, h->thermo, V.P, V.f[F_THL_H], V.f[F_QT_H], nullptr, nullptr, nullptr,
                     nullptr, V.f[F_B_H], V.f[F_QL_M], V.f[F_CPMPI_M], nullptr, s);
    const T *lag = nullptr;
    for (int k = 0; k < K; ++k) {
      const T *thm = V.f[F_THL_H], *qtm = V.f[F_QT_H], *bm = V.f[F_B_H];
      if (k > 0) {
        launch_thermo<T>(g, h->thermo, V.P, V.thl, V.qt, V.f[F_THL_H], V.f[F_QT_H], V.f[F_THL_M],
                         V.f[F_QT_M], V.f[F_B_M], V.f[F_QL_M], V.f[F_CPMPI_M], nullptr, s);
        thm = V.f[F_THL_M];
        qtm = V.f[F_QT_M];
        bm = V.f[F_B_M];
      }
      launch_radiation<T>(g, V.P, c.rad_F0, c.rad_kappa, V.f[F_QL_M], V.f[F_CPMPI_M], V.f[F_RAD], s);
      launch_sgs_nu<T>(g, V.dyn, V.u, V.v, V.w, bm, V.f[F_NU_S], s);
      launch_scalar_update<T>(g, V.dyn, V.P, V.u, V.v, V.w, thm, qtm, V.f[F_THL_H], V.f[F_QT_H],
                              V.f[F_NU_S], V.f[F_RAD], V.thl, V.qt, s);
      const T *uh = V.f[F_UN], *vh = V.f[F_VN], *wh = V.f[F_WN];
      const T *num = V.f[F_NU_S];
      if (k > 0) {
        launch_average<T>(g, V.u, V.f[F_UN], V.f[F_UH], V.v, V.f[F_VN], V.f[F_VH], V.w, V.f[F_WN],
                          V.f[F_WH], s);
        launch_sgs_nu<T>(g, V.dyn, V.f[F_UH], V.f[F_VH], V.f[F_WH], V.f[F_B_H], V.f[F_NU_M], s);
        uh = V.f[F_UH];
        vh = V.f[F_VH];
        wh = V.f[F_WH];
        num = V.f[F_NU_M];
      }
      launch_momentum<T>(g, V.dyn, V.P, uh, vh, wh, V.f[F_UN], V.f[F_VN], V.f[F_WN], V.p,
                         V.f[F_B_H], num, V.u, V.v, V.w, s);
      launch_poisson_rhs<T>(g, V.dyn, V.P, V.u, V.v, V.w, lag, V.f[F_RHS], V.partials, s);
      LAUNCH_TRY();
      const int solve_idx = step * K + k;
      const int fixed = opts && opts->replay_sweeps ? opts->replay_sweeps[solve_idx] : 0;
      if (opts && opts->replay_sweeps && fixed < 0)
        return fail(LES_ERR_ARG, "replay_sweeps[%d] = %d < 0", solve_idx, fixed);
      // the solve's time includes preparing its right-hand side and guess
      HIP_TRY(hipEventRecord(h->ev_s0, s));
      int rc = prepare_rhs<T>(h, V, V.f[F_RHS], fixed > 0 ? fixed : c.poisson_max_sweeps,
                              fixed > 0);
      if (rc) return rc;
      // Starting iterate: the previous step's solution of this sub-iteration
      // (corrected by the network in the learned form, whose input is the
      // residual of that solution for the centred right-hand side), or at
      // k = 0 the extrapolated pressure change alpha0 (p^n - p^{n-1}): p
      // holds p^n and the workspace p^{n-1}, then p^{n-1} <- p^n (corrected
      // by the three-input network in LES_GUESS_LEARNED3).  `base`: the
      // field a guess starts from (dumped for training pairs).
      T *hist = (T *)ws(h, h->lay.hist) + (size_t)k * g.n;
      const T *guess = nullptr, *base = nullptr;
      if (uses_hist(&c)) {
        if (h->hist_valid[k]) {
          base = hist;
          if (c.guess == LES_GUESS_PREVIOUS) {
            guess = hist;
          } else {
            int grc = cnn_guess<T>(h, V, V.f[F_RHS], hist, V.f[F_GUESS]);
            // further passes correct the guess from its own residual (in
            // place: each output cell reads only its own base value)
            for (int pass = 1; grc == 0 && pass < c.guess_passes; ++pass)
              grc = cnn_guess<T>(h, V, V.f[F_RHS], V.f[F_GUESS], V.f[F_GUESS]);
            if (grc) return grc;
            guess = V.f[F_GUESS];
          }
        }
      } else if (k == 0 && uses_pm2(&c)) {
        T *ext = c.guess == LES_GUESS_EXTRAPOLATE ? V.f[F_GUESS] : hist;
        launch_extrapolate<T>(g, V.P, V.p, V.f[F_PM2], ext, s);
        HIP_TRY(hipMemcpyAsync(V.f[F_PM2], V.p, bytes, hipMemcpyDeviceToDevice, s));
        LAUNCH_TRY();
        base = guess = ext;
        if (c.guess == LES_GUESS_LEARNED3) {
          const int grc = cnn_guess<T>(h, V, V.f[F_RHS], ext, V.f[F_GUESS]);
          if (grc) return grc;
          guess = V.f[F_GUESS];
        }
      }
      if (step == nsteps - 1 && opts && opts->dump_base) {
        T *db = (T *)opts->dump_base + (size_t)k * g.n;
        if (base)
          HIP_TRY(hipMemcpyAsync(db, base, bytes, hipMemcpyDeviceToDevice, s));
        else
          launch_zero<T>(g, db, s);
      }
      // Defect form: the sweeps solve for the correction from zero, so FP32
      // rounding acts at the correction's size, not the guess's.  A guess
      // whose residual is not below the zero start's is dropped.
      if (guess && (rc = prepare_guess<T>(h, V, guess, false))) return rc;
      les_solve_stats st;
      T *phi = nullptr;
      SweepTiming timing;
      timing.enabled = opts && opts->time_sweeps;
      rc = solve_prepared<T>(h, V, guess, true, fixed, h->zero_sweeps[k], &st, &phi, &timing);
      if (rc >= 0) {  // the last count of a pass from the zero start: the next guess's budget
        if (st.guess == 0 || st.guess == 2) h->zero_sweeps[k] = st.sweeps;
        else if (st.guess == 3) h->zero_sweeps[k] = st.sweeps - st.guess_sweeps;
      }
      acc.sweep_seconds += timing.seconds;
      acc.sweeps_timed += timing.sweeps;
      if (opts && opts->records) opts->records[solve_idx] = st;
      if (rc < 0) return rc;
      acc.solves++;
      acc.sweeps_total += st.sweeps;
      if (st.sweeps > acc.sweeps_max) acc.sweeps_max = st.sweeps;
      if (st.status == 1) {
        acc.not_converged++;
        rc_final = LES_WARN_NOT_CONVERGED;
      }
      const double rel = st.rhs_norm > 0 ? st.res_norm / st.rhs_norm : 0.0;
      if (rel > acc.res_rel_max) acc.res_rel_max = rel;
      acc.poisson_seconds += st.seconds;
      // gauge (zero mean); profile terms of the horizontally uniform part
      // (projection, the next sub-iteration's right-hand side) and its
      // pressure, p_bar += rho0 phi_bar in FP64
      launch_block_sum<T>(phi, g.n, 0, V.partials, s);
      launch_final(V.partials, kReduceBlocks, kFinalPhiMean, V.ctl, (double)g.n, 0.0, 0, nullptr, s);
      launch_mean_profiles<T>(g, V.phibar, V.P.rho0, V.P.alpha0, 1, V.pbar, V.phigz_w, V.cbar_w,
                              V.pgz_w, s);
      if (uses_hist(&c)) {
        launch_sub_mean<T>(g, phi, V.ctl, hist, s);
        h->hist_valid[k] = 1;
      }
      if (step == nsteps - 1 && opts) {  // the last step's solves (training pairs)
        if (opts->dump_rhs)
          HIP_TRY(hipMemcpyAsync((T *)opts->dump_rhs + (size_t)k * g.n, V.f[F_RHS], bytes,
                                 hipMemcpyDeviceToDevice, s));
        if (opts->dump_phi)
          launch_sub_mean<T>(g, phi, V.ctl, (T *)opts->dump_phi + (size_t)k * g.n, s);
        if (opts->dump_mean) {
          // per-level values the centring removed and the solution's
          // horizontally uniform part (FP64, host)
          double *dm = opts->dump_mean + (size_t)k * (2 * g.nz + 1);
          HIP_TRY(hipMemcpyAsync(dm, V.rsub, g.nz * sizeof(double), hipMemcpyDeviceToHost, s));
          HIP_TRY(hipMemcpyAsync(dm + g.nz, V.phibar, g.nz * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
          HIP_TRY(hipMemcpyAsync(dm + 2 * g.nz, &V.ctl->rhs_mean, sizeof(double),
                                 hipMemcpyDeviceToHost, s));
          HIP_TRY(hipStreamSynchronize(s));
        }
      }
      launch_project<T>(g, V.dyn, V.P, phi, V.ctl, V.u, V.v, V.w, V.p, s);
      LAUNCH_TRY();
      lag = phi;
    }
    acc.steps++;
    h->steps_done++;
  }
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  acc.seconds = ms * 1e-3;
  if (stats) *stats = acc;
  return rc_final;
}

template <typename T>
int poisson_impl(les_handle *h, const void *rhs, void *phi, const les_poisson_opts *opts,
                 les_solve_stats *stats) {
  View<T> V = view_of<T>(h);
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  const int use_guess = opts ? opts->use_guess : 0;
  const int fixed = opts ? opts->fixed_sweeps : 0;
  if (fixed < 0) return fail(LES_ERR_ARG, "fixed_sweeps < 0");
  if (use_guess < 0 || use_guess > 2) return fail(LES_ERR_ARG, "use_guess must be 0, 1 or 2");
  HIP_TRY(hipEventRecord(h->ev_s0, s));
  int rc = prepare_rhs<T>(h, V, (const T *)rhs, fixed > 0 ? fixed : h->cfg.poisson_max_sweeps,
                          fixed > 0);
  if (rc) return rc;
  const T *guess = nullptr;
  if (use_guess) {
    HIP_TRY(hipMemcpyAsync(V.f[F_GUESS], phi, (size_t)g.n * sizeof(T), hipMemcpyDeviceToDevice,
                           s));
    guess = V.f[F_GUESS];
    if ((rc = prepare_guess<T>(h, V, guess, use_guess == 1))) return rc;
  }
  les_solve_stats st;
  T *res = nullptr;
  const int budget = opts ? opts->budget : 0;
  if (budget < 0) return fail(LES_ERR_ARG, "budget < 0");
  rc = solve_prepared<T>(h, V, guess, use_guess == 2, fixed, budget, &st, &res, nullptr);
  if (stats) *stats = st;
  if (rc < 0) return rc;
  launch_block_sum<T>(res, g.n, 0, V.partials, s);
  launch_final(V.partials, kReduceBlocks, kFinalPhiMean, V.ctl, (double)g.n, 0.0, 0, nullptr, s);
  launch_add_profile<T>(g, res, V.ctl, V.phibar, (T *)phi, s);
  LAUNCH_TRY();
  HIP_TRY(hipStreamSynchronize(s));
  return st.status == 1 ? LES_WARN_NOT_CONVERGED : LES_OK;
}

// The momentum predictor's profile d_c(alpha0 pbar)/dz from the pbar held
// in the workspace.  Synchronizes.
template <typename T>
int set_pressure_profile_device(les_handle *h) {
  View<T> V = view_of<T>(h);
  launch_mean_profiles<T>(h->grid, nullptr, V.P.rho0, V.P.alpha0, 0, V.pbar, V.phigz_w, V.cbar_w,
                          V.pgz_w, h->stream);
  LAUNCH_TRY();
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LES_OK;
}

template <typename T>
int set_pressure_profile_impl(les_handle *h, const double *pbar_host) {
  View<T> V = view_of<T>(h);
  HIP_TRY(hipMemcpyAsync(V.pbar, pbar_host, h->grid.nz * sizeof(double), hipMemcpyHostToDevice,
                         h->stream));
  return set_pressure_profile_device<T>(h);
}

template <typename T>
int pressure_impl(les_handle *h, void *p_out, double *pbar_host) {
  View<T> V = view_of<T>(h);
  if (p_out) launch_add_profile<T>(h->grid, V.p, nullptr, V.pbar, (T *)p_out, h->stream);
  LAUNCH_TRY();
  if (pbar_host)
    HIP_TRY(hipMemcpyAsync(pbar_host, V.pbar, h->grid.nz * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LES_OK;
}

template <typename T>
int thermo_impl(les_handle *h, const void *thl, const void *qt, void *Tout, void *ql, void *b) {
  View<T> V = view_of<T>(h);
  launch_thermo<T>(h->grid, h->thermo, V.P, (const T *)thl, (const T *)qt, nullptr, nullptr,
                   nullptr, nullptr, (T *)b, (T *)ql, nullptr, (T *)Tout, h->stream);
  LAUNCH_TRY();
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LES_OK;
}

template <typename T>
int diag_impl(les_handle *h, les_diag *out, double *profiles) {
  View<T> V = view_of<T>(h);
  const Grid &g = h->grid;
  const int nz = g.nz;
  launch_thermo<T>(g, h->thermo, V.P, V.thl, V.qt, nullptr, nullptr, nullptr, nullptr,
                   V.f[F_B_M], V.f[F_QL_M], nullptr, nullptr, h->stream);
  launch_diag<T>(g, V.dyn, V.P, V.u, V.v, V.w, V.thl, V.qt, V.f[F_QL_M], V.f[F_B_M], V.diag,
                 h->stream);
  LAUNCH_TRY();
  HIP_TRY(hipMemcpyAsync(h->diag_host, V.diag, (size_t)nz * kDiagStride * sizeof(double),
                         hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const double *L = h->diag_host;
  const double dV = g.dx * g.dy * g.dz;
  les_diag d;
  std::memset(&d, 0, sizeof(d));
  double div2 = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double *r = L + (size_t)k * kDiagStride;
    d.mass_thl += r[9] * dV;
    d.mass_qt += r[10] * dV;
    d.ke += r[11] * dV;
    div2 += r[12];
    d.div_max = r[13] > d.div_max ? r[13] : d.div_max;
    d.cfl = r[14] > d.cfl ? r[14] : d.cfl;
    if (profiles)
      for (int m = 0; m < LES_NPROFILES; ++m) profiles[(size_t)m * nz + k] = r[m] / (double)g.nxy;
  }
  d.div_l2 = std::sqrt(div2);
  if (out) *out = d;
  return LES_OK;
}

// Learned guess: r = rhs - L base, s = RMS(r) (FP64 sums), network on
// bf16(r / s) (three inputs: and bf16(base d / s), bf16(rhs / s)) over the
// periodic field, guess = base + (s/d) out.
template <typename T>
int cnn_guess(les_handle *h, View<T> &V, const T *rhs, const T *base, T *guess) {
  if (!h->cnn_bound)
    return fail(LES_ERR_STATE, "learned guess requested but no network is bound (les_bind_cnn)");
  const Grid &g = h->grid;
  hipStream_t s = h->stream;
  const Layout &L = h->lay;
  float *r = (float *)ws(h, L.cnn_r);
  uint16_t *a0 = (uint16_t *)ws(h, L.cnn_a0);
  uint16_t *act[2] = {(uint16_t *)ws(h, L.cnn_act[0]), (uint16_t *)ws(h, L.cnn_act[1])};
  const float *params = (const float *)ws(h, L.cnn_params);
  const uint16_t *packed = (const uint16_t *)ws(h, L.cnn_packed);
  double *sc = (double *)ws(h, L.cnn_sc);
  const double D = 2.0 / (g.dx * g.dx) + 2.0 / (g.dy * g.dy) + 2.0 / (g.dz * g.dz);
  const int ci = cnn_inputs_of(&h->cfg);
  launch_cnn_residual<T>(g, rhs, base, r, V.partials, s);
  launch_cnn_scale(V.partials, (double)g.n, D, sc, s);
  // one periodic field: batch 1, (nz, ny, nx)
  auto geom = [&](int l) { return cnn_geom(1, g.nz, g.ny, g.nx, 1, l, ci); };
  if (ci == 3) {
    launch_cnn_input3<T>(g, r, base, rhs, sc, D, a0, s);
    launch_cnn_conv(0, geom(0), a0, params, packed, h->cnn_alpha, act[0], nullptr, s);
    launch_cnn_conv(1, geom(1), act[0], params, packed, h->cnn_alpha, act[1], nullptr, s);
  } else {  // the input r / s is rounded inside the fused first two layers
    launch_cnn_in_mid(geom(1), r, sc + 1, params, packed, h->cnn_alpha, act[1], s);
  }
  launch_cnn_conv(2, geom(2), act[1], params, packed, h->cnn_alpha, act[0], nullptr, s);
  launch_cnn_guess<T>(geom(3), act[0], params, packed, base, sc + 2, guess, s);
  LAUNCH_TRY();
  return LES_OK;
}

// Exported state: a header, then the FP64 pressure profile, then (by guess
// mode) the previous step's pressure or the previous step's solutions of
// each sub-iteration, each region 256-byte aligned.
struct StateHeader {
  char magic[8];  // "LESSTAT1"
  int32_t nx, ny, nz, precision, mean_mode, guess, n_subiter, reserved;
  uint64_t hist_valid;  // bit k: sub-iteration k's previous solution is held
  int64_t steps_done;
};
static_assert(sizeof(StateHeader) <= kAlign, "state header exceeds its region");

struct StateLayout {
  size_t zsw, pbar, pm2, hist, total;
};

StateLayout state_layout(const les_config &c) {
  const size_t n = (size_t)c.nx * c.ny * c.nz, es = elem_size(&c);
  StateLayout S;
  size_t off = kAlign;
  S.zsw = off;  // n_subiter int32: the guesses' sweep budgets
  off = align_up(off + (size_t)c.n_subiter * sizeof(int32_t));
  S.pbar = off;
  off = align_up(off + (size_t)c.nz * sizeof(double));
  S.pm2 = off;
  if (uses_pm2(&c)) off = align_up(off + n * es);
  S.hist = off;
  if (uses_hist(&c)) off = align_up(off + (size_t)c.n_subiter * n * es);
  S.total = off;
  return S;
}

int check_handle(const les_handle *h) {
  if (!h) return fail(LES_ERR_ARG, "handle is NULL");
  if (h->broken) return fail(LES_ERR_STATE, "handle unusable after an earlier HIP error");
  return LES_OK;
}

}  // namespace

extern "C" {

void les_default_config(les_config *c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->nx = c->ny = c->nz = 32;
  c->precision = LES_FP64;
  c->n_subiter = 2;
  c->poisson_scheme = LES_JACOBI;
  c->poisson_check_every = 25;
  c->poisson_max_sweeps = 200000;
  c->satadj_maxit = 20;
  c->dx = c->dy = 40.0;
  c->dz = 10.0;
  c->dt = 0.5;
  c->poisson_tol = 1e-8;
  c->jacobi_omega = 0.0;
  // Table 1 of the paper
  c->p00 = 1.0e5;
  c->theta0 = 290.0;
  c->Rd = 287.0;
  c->Rv = 461.89;
  c->cpd = 1004.5;
  c->cpv = 1859.5;
  c->cl = 4181.0;
  c->ci = 2100.0;
  c->Lv0 = 2.47e6;
  c->Ls0 = 2.83e6;
  c->Tf = 273.15;
  c->fcor = 7.62e-5;
  c->g = 9.81;
  c->cs = 0.18;
  c->Pr = 0.4;
  c->Sc = 0.4;
  c->ug = 7.0;
  c->vg = -5.0;
  c->sponge_frac = 0.05;
  c->sponge_max = 0.25;
  c->e_tr = 611.657;
  c->T_tr = 273.16;
  c->satadj_tol = 1e-10;
  c->T_ice = 233.15;
  c->mean_mode = LES_MEAN_EXACT;
}

size_t les_workspace_bytes(const les_config *cfg) {
  if (validate(cfg) != LES_OK) return 0;
  return layout_of(cfg).total;
}

int les_workspace_offset(const les_config *cfg, int32_t field, size_t *offset) {
  int rc = validate(cfg);
  if (rc) return rc;
  if (field < 0 || field >= F_COUNT || !offset) return fail(LES_ERR_ARG, "unknown field %d", field);
  *offset = layout_of(cfg).field[field];
  return LES_OK;
}

namespace {
int init_impl(const les_config *cfg, const les_buffers *bufs, void *stream, les_handle **out);
}

int les_init(const les_config *cfg, const les_buffers *bufs, void *stream, les_handle **out) {
  if (out) *out = nullptr;
  return guarded([&] { return init_impl(cfg, bufs, stream, out); });
}

}  // extern "C"

namespace {

int init_impl(const les_config *cfg, const les_buffers *bufs, void *stream, les_handle **out) {
  if (!out) return fail(LES_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  if (!bufs) return fail(LES_ERR_ARG, "buffers are NULL");
  const size_t es = elem_size(cfg);
  void *const ptrs[7] = {bufs->u, bufs->v, bufs->w, bufs->thl, bufs->qt, bufs->p, bufs->workspace};
  const char *names[7] = {"u", "v", "w", "thl", "qt", "p", "workspace"};
  for (int q = 0; q < 7; ++q) {
    if (!ptrs[q]) return fail(LES_ERR_ARG, "buffer %s is NULL", names[q]);
    if ((uintptr_t)ptrs[q] % (q == 6 ? kAlign : es))
      return fail(LES_ERR_ARG, "buffer %s is misaligned", names[q]);
  }
  const Layout L = layout_of(cfg);
  if (bufs->workspace_bytes < L.total)
    return fail(LES_ERR_ARG, "workspace has %zu bytes, needs %zu", bufs->workspace_bytes, L.total);

  les_handle *h = new les_handle();
  h->cfg = *cfg;
  h->buf = *bufs;
  h->stream = (hipStream_t)stream;
  h->lay = L;
  h->broken = false;
  Grid &g = h->grid;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->nz;
  g.nxy = (int64_t)cfg->nx * cfg->ny;
  g.sy = cfg->ny == 1 ? 0 : cfg->nx;
  g.n = g.nxy * cfg->nz;
  g.dx = cfg->dx;
  g.dy = cfg->dy;
  g.dz = cfg->dz;
  g.dt = cfg->dt;
  Thermo &t = h->thermo;
  t.p00 = cfg->p00;
  t.Rd = cfg->Rd;
  t.Rv = cfg->Rv;
  t.cpd = cfg->cpd;
  t.cpv = cfg->cpv;
  t.cl = cfg->cl;
  t.ci = cfg->ci;
  t.Lv0 = cfg->Lv0;
  t.Ls0 = cfg->Ls0;
  t.Tf = cfg->Tf;
  t.g = cfg->g;
  t.e_tr = cfg->e_tr;
  t.inv_Ttr = 1.0 / cfg->T_tr;
  t.Lv_over_Rv = cfg->Lv0 / cfg->Rv;
  t.Ls_over_Rv = cfg->Ls0 / cfg->Rv;
  t.eps = cfg->Rd / cfg->Rv;
  t.phase = cfg->phase;
  t.T_ice = cfg->T_ice;
  t.inv_ramp = cfg->phase == LES_PHASE_RAMP ? 1.0 / (cfg->Tf - cfg->T_ice) : 0.0;
  t.satadj_tol = cfg->satadj_tol;
  t.satadj_maxit = cfg->satadj_maxit;
  jacobi_spectrum(cfg, &h->mu_min, &h->mu_max);
  h->hist_valid.assign(cfg->n_subiter, 0);
  h->zero_sweeps.assign(cfg->n_subiter, 0);
  h->cnn_bound = false;
  h->cnn_alpha = 0.f;
  h->steps_done = 0;
  h->sweeps_per_launch = cfg->sweeps_per_launch > 0 ? cfg->sweeps_per_launch : kDefaultSweepsPerLaunch;

  auto cleanup = [&](int code) {
    les_destroy(h);
    return code;
  };
  if (hipHostMalloc((void **)&h->ctl_host, 8 * sizeof(SolveCtl), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(LES_ERR_HIP, "hipHostMalloc failed"));
  // residual-test word: written by kernels, read by the host while they run,
  // so coherent, mapped host memory seen through its device pointer
  if (hipHostMalloc((void **)&h->poll_word, 256, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return cleanup(fail(LES_ERR_HIP, "hipHostMalloc (coherent) failed"));
  std::memset(h->poll_word, 0, 256);
  if (hipHostGetDevicePointer((void **)&h->poll_word_dev, h->poll_word, 0) != hipSuccess)
    return cleanup(fail(LES_ERR_HIP, "hipHostGetDevicePointer failed"));
  if (hipHostMalloc((void **)&h->diag_host, (size_t)cfg->nz * kDiagStride * sizeof(double),
                    hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(LES_ERR_HIP, "hipHostMalloc failed"));
  if (hipEventCreate(&h->ev_s0) != hipSuccess || hipEventCreate(&h->ev_s1) != hipSuccess ||
      hipEventCreate(&h->ev_a) != hipSuccess || hipEventCreate(&h->ev_b) != hipSuccess)
    return cleanup(fail(LES_ERR_HIP, "hipEventCreate failed"));
  rc = cfg->precision == LES_FP64 ? upload_profiles<double>(h) : upload_profiles<float>(h);
  if (!rc && hipMemcpyAsync(ws(h, L.field[F_PM2]), bufs->p, (size_t)g.n * es,
                            hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
    rc = fail(LES_ERR_HIP, "copy of the initial pressure failed");
  if (!rc && hipStreamSynchronize(h->stream) != hipSuccess)
    rc = fail(LES_ERR_HIP, "hipStreamSynchronize failed");
  if (rc) return cleanup(rc);
  *out = h;
  return LES_OK;
}

}  // namespace

extern "C" {

int les_step(les_handle *h, int32_t nsteps, const les_step_opts *opts, les_step_stats *stats) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (nsteps < 0) return fail(LES_ERR_ARG, "nsteps < 0");
  rc = guarded([&] {
    return h->cfg.precision == LES_FP64 ? step_impl<double>(h, nsteps, opts, stats)
                                        : step_impl<float>(h, nsteps, opts, stats);
  });
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

int les_poisson_solve(les_handle *h, const void *rhs, void *phi, const les_poisson_opts *opts,
                      les_solve_stats *stats) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!rhs || !phi) return fail(LES_ERR_ARG, "rhs and phi must be non-NULL");
  rc = guarded([&] {
    return h->cfg.precision == LES_FP64 ? poisson_impl<double>(h, rhs, phi, opts, stats)
                                        : poisson_impl<float>(h, rhs, phi, opts, stats);
  });
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

size_t les_state_bytes(const les_handle *h) {
  if (!h) return 0;
  return state_layout(h->cfg).total;
}

int les_export_state(les_handle *h, void *dst) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!dst) return fail(LES_ERR_ARG, "dst is NULL");
  if ((uintptr_t)dst % kAlign) return fail(LES_ERR_ARG, "dst is not 256-byte aligned");
  const les_config &c = h->cfg;
  const StateLayout S = state_layout(c);
  const size_t n = (size_t)h->grid.n, es = elem_size(&c);
  StateHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, "LESSTAT1", 8);
  hd.nx = c.nx;
  hd.ny = c.ny;
  hd.nz = c.nz;
  hd.precision = c.precision;
  hd.mean_mode = c.mean_mode;
  hd.guess = c.guess;
  hd.n_subiter = c.n_subiter;
  for (int k = 0; k < c.n_subiter; ++k)
    if (h->hist_valid[k]) hd.hist_valid |= (uint64_t)1 << k;
  hd.steps_done = h->steps_done;
  char *d = (char *)dst;
  auto copy = [&](void *to, const void *from, size_t bytes, hipMemcpyKind kind) {
    return hipMemcpyAsync(to, from, bytes, kind, h->stream);
  };
  hipError_t e = copy(d, &hd, sizeof(hd), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = copy(d + S.zsw, h->zero_sweeps.data(), (size_t)c.n_subiter * sizeof(int32_t),
             hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = copy(d + S.pbar, ws(h, h->lay.mean_d) + pbar_index(c.nz) * sizeof(double),
             (size_t)c.nz * sizeof(double), hipMemcpyDeviceToDevice);
  if (e == hipSuccess && uses_pm2(&c))
    e = copy(d + S.pm2, ws(h, h->lay.field[F_PM2]), n * es, hipMemcpyDeviceToDevice);
  if (e == hipSuccess && uses_hist(&c))
    e = copy(d + S.hist, ws(h, h->lay.hist), (size_t)c.n_subiter * n * es,
             hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "exporting the state failed: %s", hipGetErrorString(e));
  }
  return LES_OK;
}

int les_import_state(les_handle *h, const void *src) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!src) return fail(LES_ERR_ARG, "src is NULL");
  const les_config &c = h->cfg;
  const StateLayout S = state_layout(c);
  const size_t n = (size_t)h->grid.n, es = elem_size(&c);
  StateHeader hd;
  if (hipMemcpyAsync(&hd, src, sizeof(hd), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "reading the state header failed");
  }
  if (std::memcmp(hd.magic, "LESSTAT1", 8) != 0)
    return fail(LES_ERR_ARG, "src does not hold an exported state");
  if (hd.nx != c.nx || hd.ny != c.ny || hd.nz != c.nz || hd.precision != c.precision ||
      hd.mean_mode != c.mean_mode || hd.guess != c.guess || hd.n_subiter != c.n_subiter)
    return fail(LES_ERR_ARG,
                "state of a %dx%dx%d grid (precision %d, mean mode %d, guess %d, K %d) does not "
                "match this handle",
                hd.nx, hd.ny, hd.nz, hd.precision, hd.mean_mode, hd.guess, hd.n_subiter);
  const char *d = (const char *)src;
  auto copy = [&](void *to, const void *from, size_t bytes) {
    return hipMemcpyAsync(to, from, bytes, hipMemcpyDeviceToDevice, h->stream);
  };
  hipError_t e = copy(ws(h, h->lay.mean_d) + pbar_index(c.nz) * sizeof(double), d + S.pbar,
                      (size_t)c.nz * sizeof(double));
  if (e == hipSuccess && uses_pm2(&c))
    e = copy(ws(h, h->lay.field[F_PM2]), d + S.pm2, n * es);
  if (e == hipSuccess && uses_hist(&c))
    e = copy(ws(h, h->lay.hist), d + S.hist, (size_t)c.n_subiter * n * es);
  if (e != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "importing the state failed: %s", hipGetErrorString(e));
  }
  // the momentum predictor's pressure-gradient profile follows the profile
  rc = c.precision == LES_FP64 ? set_pressure_profile_device<double>(h)
                               : set_pressure_profile_device<float>(h);
  if (rc) {
    if (rc == LES_ERR_HIP) h->broken = true;
    return rc;
  }
  std::vector<int32_t> zsw(c.n_subiter);
  if (hipMemcpyAsync(zsw.data(), d + S.zsw, (size_t)c.n_subiter * sizeof(int32_t),
                     hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "reading the guess budgets failed");
  }
  for (int k = 0; k < c.n_subiter; ++k) h->hist_valid[k] = (hd.hist_valid >> k) & 1;
  h->zero_sweeps = zsw;
  h->steps_done = hd.steps_done;
  return LES_OK;
}

int64_t les_steps_done(const les_handle *h) { return h ? h->steps_done : -1; }

int les_set_pressure_profile(les_handle *h, const double *pbar_host) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!pbar_host) return fail(LES_ERR_ARG, "pbar_host is NULL");
  if (h->cfg.mean_mode == LES_MEAN_SWEPT)
    return fail(LES_ERR_STATE, "les_set_pressure_profile needs LES_MEAN_LEVEL or LES_MEAN_EXACT");
  for (int k = 0; k < h->cfg.nz; ++k)
    if (!std::isfinite(pbar_host[k])) return fail(LES_ERR_ARG, "pbar_host[%d] is not finite", k);
  rc = h->cfg.precision == LES_FP64 ? set_pressure_profile_impl<double>(h, pbar_host)
                                    : set_pressure_profile_impl<float>(h, pbar_host);
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

int les_pressure(les_handle *h, void *p_out, double *pbar_host) {
  int rc = check_handle(h);
  if (rc) return rc;
  rc = h->cfg.precision == LES_FP64 ? pressure_impl<double>(h, p_out, pbar_host)
                                    : pressure_impl<float>(h, p_out, pbar_host);
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

int les_thermo(les_handle *h, const void *thl, const void *qt, void *T, void *ql, void *b) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!thl || !qt) return fail(LES_ERR_ARG, "thl and qt must be non-NULL");
  rc = h->cfg.precision == LES_FP64 ? thermo_impl<double>(h, thl, qt, T, ql, b)
                                    : thermo_impl<float>(h, thl, qt, T, ql, b);
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

int les_diagnostics(les_handle *h, les_diag *out, double *profiles) {
  int rc = check_handle(h);
  if (rc) return rc;
  rc = h->cfg.precision == LES_FP64 ? diag_impl<double>(h, out, profiles)
                                    : diag_impl<float>(h, out, profiles);
  if (rc == LES_ERR_HIP) h->broken = true;
  return rc;
}

void les_destroy(les_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->ev_s0) (void)hipEventDestroy(h->ev_s0);
  if (h->ev_s1) (void)hipEventDestroy(h->ev_s1);
  if (h->ev_a) (void)hipEventDestroy(h->ev_a);
  if (h->ev_b) (void)hipEventDestroy(h->ev_b);
  for (auto &e : h->ev_sweep) (void)hipEventDestroy(e);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  if (h->poll_word) (void)hipHostFree(h->poll_word);
  if (h->diag_host) (void)hipHostFree(h->diag_host);
  delete h;
}

int les_bind_cnn(les_handle *h, const float *params, double alpha) {
  int rc = check_handle(h);
  if (rc) return rc;
  const int ci = cnn_inputs_of(&h->cfg);
  if (!ci)
    return fail(LES_ERR_STATE,
                "les_bind_cnn: the handle was not created with LES_GUESS_LEARNED or _LEARNED3");
  if (!params) return fail(LES_ERR_ARG, "params is NULL");
  if (!(alpha >= 0.0)) return fail(LES_ERR_ARG, "alpha must be >= 0");
  float *dst = (float *)ws(h, h->lay.cnn_params);
  if (hipMemcpyAsync(dst, params, (size_t)cnn_param_count(ci) * sizeof(float),
                     hipMemcpyDeviceToDevice, h->stream) != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "copy of the network parameters failed");
  }
  launch_cnn_pack(dst, cnn_param_count(ci), (uint16_t *)ws(h, h->lay.cnn_packed), h->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    h->broken = true;
    return fail(LES_ERR_HIP, "packing the network parameters failed");
  }
  h->cnn_bound = true;
  h->cnn_alpha = (float)alpha;
  return LES_OK;
}

int les_cnn_guess(les_handle *h, const void *rhs, const void *base, void *guess, double *scale) {
  int rc = check_handle(h);
  if (rc) return rc;
  if (!cnn_inputs_of(&h->cfg))
    return fail(LES_ERR_STATE,
                "les_cnn_guess: the handle was not created with LES_GUESS_LEARNED or _LEARNED3");
  if (!rhs || !base || !guess) return fail(LES_ERR_ARG, "rhs, base and guess must be non-NULL");
  if (h->cfg.precision == LES_FP64) {
    View<double> V = view_of<double>(h);
    rc = cnn_guess<double>(h, V, (const double *)rhs, (const double *)base, (double *)guess);
  } else {
    View<float> V = view_of<float>(h);
    rc = cnn_guess<float>(h, V, (const float *)rhs, (const float *)base, (float *)guess);
  }
  if (rc) {
    if (rc == LES_ERR_HIP) h->broken = true;
    return rc;
  }
  if (scale) {
    if (hipMemcpyAsync(scale, ws(h, h->lay.cnn_sc), sizeof(double), hipMemcpyDeviceToHost,
                       h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
      h->broken = true;
      return fail(LES_ERR_HIP, "reading the guess scale failed");
    }
  }
  return LES_OK;
}

const char *les_last_error(void) { return g_error.c_str(); }

}  // extern "C"
