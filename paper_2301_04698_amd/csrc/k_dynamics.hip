// Subgrid viscosity (paper Sec. 2.3), scalar predictor (Sec. 2.4, scalar
// prediction equation) and momentum predictor (Sec. 2.4, momentum
// prediction equation) on the collocated grid.  One thread per cell; the
// stencil neighbourhoods are served by the L1/L2 caches.
#include "les.h"
#include "les_device.h"

namespace lesmi {

namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

struct Cell {
  int i, j, k;
};

__device__ __forceinline__ Cell cell_of(const Grid &g, int64_t q) {
  const int k = (int)(q / g.nxy);
  const int64_t r = q - g.nxy * k;
  const int j = (int)(r / g.nx);
  return Cell{(int)(r - (int64_t)g.nx * j), j, k};
}

// QUICK face value at l+1/2 from q(l-1), q(l), q(l+1), q(l+2), upwinded on
// the face mass flux m (Leonard's quadratic upstream interpolation).
template <typename T>
__device__ __forceinline__ T quick(T m, T qm1, T q0, T q1, T q2) {
  return m >= T(0) ? (T(6) * q0 + T(3) * q1 - qm1) / T(8) : (T(6) * q1 + T(3) * q0 - q2) / T(8);
}

// Third-order WENO face value at l+1/2 taken from the upwind side, from
// a = q(l-1), b = q(l), c = q(l+1): candidates (-a + 3b)/2 and (b + c)/2,
// linear weights 1/3 and 2/3, smoothness (b - a)^2 and (c - b)^2 (Jiang &
// Shu), eps = 1e-6 max(a^2, b^2, c^2) + 1e-18 so the weights do not depend
// on the field's units; the weight is formed without small squares in a
// denominator.
template <typename T>
__device__ __forceinline__ T weno3(T a, T b, T c) {
  const T eps = T(1e-6) * max(a * a, max(b * b, c * c)) + T(1e-18);
  const T s0 = eps + (b - a) * (b - a), s1 = eps + (c - b) * (c - b);
  const T w0 = (T(1) / T(3)) * s1 * s1 / ((T(1) / T(3)) * s1 * s1 + (T(2) / T(3)) * s0 * s0);
  return w0 * (-a + T(3) * b) / T(2) + (T(1) - w0) * (b + c) / T(2);
}

// Advective flux m * (face value) through face l+1/2 of the five values
// q(l-1) .. q(l+2): QUICK upwinded on m, or WENO3 with the Lax-Friedrichs
// flux at the face speed |m| (the upwind-side reconstruction; zero on the
// walls with m).
template <typename T, bool WENO>
__device__ __forceinline__ T face_flux(T m, T qm1, T q0, T q1, T q2) {
  if (WENO) {
    const T lo = weno3(qm1, q0, q1), hi = weno3(q2, q1, q0);
    return T(0.5) * m * (lo + hi) - T(0.5) * fabs(m) * (hi - lo);
  }
  return m * quick(m, qm1, q0, q1, q2);
}

// Wall parity of velocity component a: w is odd across the walls (zero
// mass flux); u and v are odd for no-slip walls, even for free-slip (FS)
// ones.  A compile-time sign keeps the ghost negation free.
template <typename T, bool FS>
__device__ __forceinline__ T vpar(int a) {
  return a < 2 && FS ? T(1) : T(-1);
}

// Central derivative of velocity component a (field f) along axis ax at
// cell (i, j, k), which may be a ghost level.
template <typename T, bool FS>
__device__ __forceinline__ T dcentral(const T *__restrict__ f, const Grid &g, const Dyn<T> &d,
                                      int a, int ax, int i, int j, int k) {
  const int di = ax == 0, dj = ax == 1, dk = ax == 2;
  const T inv2 = ax == 0 ? d.inv_2dx : (ax == 1 ? d.inv_2dy : d.inv_2dz);
  const T par = vpar<T, FS>(a);
  return (gload(f, g, i + di, j + dj, k + dk, par) - gload(f, g, i - di, j - dj, k - dk, par)) *
         inv2;
}

// ---------------------------------------------------------------- SGS nu

// nu_t = (c_s Delta)^2 f_B S with S = sqrt(2 S_ij S_ij) and the buoyancy
// factor f_B = sqrt(clamp(1 - N^2/(Pr S^2), 0, 1)), N^2 = db/dz (central);
// or the uniform viscosity of the validation cases (Sec. 3) when set.
template <typename T, bool FS>
__global__ __launch_bounds__(kBlock) void sgs_nu_kernel(Grid g, Dyn<T> d, const T *__restrict__ u,
                                                        const T *__restrict__ v,
                                                        const T *__restrict__ w,
                                                        const T *__restrict__ b,
                                                        T *__restrict__ nu) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  if (d.nu_const > T(0)) {
    nu[q] = d.nu_const;
    return;
  }
  const Cell c = cell_of(g, q);
  const T *vel[3] = {u, v, w};
  T G[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int e = 0; e < 3; ++e) G[a][e] = dcentral<T, FS>(vel[a], g, d, a, e, c.i, c.j, c.k);
  T s2 = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const T sij = T(0.5) * (G[a][e] + G[e][a]);
      s2 += T(2) * sij * sij;
    }
  const T n2 = (gload(b, g, c.i, c.j, c.k + 1, T(1)) - gload(b, g, c.i, c.j, c.k - 1, T(1))) * d.inv_2dz;
  T val = T(0);
  if (s2 > T(0)) {
    T r = T(1) - n2 / (d.pr * s2);
    r = r < T(0) ? T(0) : (r > T(1) ? T(1) : r);
    val = d.smag_l2 * sqrt(s2) * sqrt(r);
  }
  nu[q] = val;
}

// ------------------------------------------------------- scalar update

// Face mass fluxes of the six faces of a cell: average of rho0 u of the
// two cells sharing the face (zero on the walls by the odd mirror of w).
template <typename T>
struct FaceFlux {
  T xm, xp, ym, yp, zm, zp;
};

template <typename T>
__device__ __forceinline__ FaceFlux<T> face_mass(const Grid &g, const Profiles<T> &P,
                                                 const T *__restrict__ u, const T *__restrict__ v,
                                                 const T *__restrict__ w, const Cell &c) {
  const T r0 = P.rho0_t[c.k];
  const T rm = pload(P.rho0_t, c.k - 1, g.nz), rp = pload(P.rho0_t, c.k + 1, g.nz);
  const T uc = r0 * gload(u, g, c.i, c.j, c.k, T(-1));
  const T vc = r0 * gload(v, g, c.i, c.j, c.k, T(-1));
  const T wc = r0 * gload(w, g, c.i, c.j, c.k, T(-1));
  FaceFlux<T> f;
  f.xp = T(0.5) * (uc + r0 * gload(u, g, c.i + 1, c.j, c.k, T(-1)));
  f.xm = T(0.5) * (r0 * gload(u, g, c.i - 1, c.j, c.k, T(-1)) + uc);
  f.yp = T(0.5) * (vc + r0 * gload(v, g, c.i, c.j + 1, c.k, T(-1)));
  f.ym = T(0.5) * (r0 * gload(v, g, c.i, c.j - 1, c.k, T(-1)) + vc);
  f.zp = T(0.5) * (wc + rp * gload(w, g, c.i, c.j, c.k + 1, T(-1)));
  f.zm = T(0.5) * (rm * gload(w, g, c.i, c.j, c.k - 1, T(-1)) + wc);
  return f;
}

// Flux-form advective tendency -div(U s) of a field s with parity par.
template <typename T, bool WENO>
__device__ __forceinline__ T advect(const Grid &g, const Dyn<T> &d, const FaceFlux<T> &f,
                                    const T *__restrict__ s, T par, const Cell &c) {
  T sx[5], sy[5], sz[5];
#pragma unroll
  for (int o = -2; o <= 2; ++o) {
    sx[o + 2] = gload(s, g, c.i + o, c.j, c.k, par);
    sy[o + 2] = gload(s, g, c.i, c.j + o, c.k, par);
    sz[o + 2] = gload(s, g, c.i, c.j, c.k + o, par);
  }
  const T fxp = face_flux<T, WENO>(f.xp, sx[1], sx[2], sx[3], sx[4]);
  const T fxm = face_flux<T, WENO>(f.xm, sx[0], sx[1], sx[2], sx[3]);
  const T fyp = face_flux<T, WENO>(f.yp, sy[1], sy[2], sy[3], sy[4]);
  const T fym = face_flux<T, WENO>(f.ym, sy[0], sy[1], sy[2], sy[3]);
  const T fzp = face_flux<T, WENO>(f.zp, sz[1], sz[2], sz[3], sz[4]);
  const T fzm = face_flux<T, WENO>(f.zm, sz[0], sz[1], sz[2], sz[3]);
  return -((fxp - fxm) * d.inv_dx + (fyp - fym) * d.inv_dy + (fzp - fzm) * d.inv_dz);
}

// Viscosity and rho0 on the six faces (means of the two adjacent cells).
template <typename T>
struct FaceVisc {
  T xm, xp, ym, yp, zm, zp;  // rho0_f * nu_f
};

template <typename T>
__device__ __forceinline__ FaceVisc<T> face_visc(const Grid &g, const Profiles<T> &P,
                                                 const T *__restrict__ nu, const Cell &c) {
  const T r0 = P.rho0_t[c.k];
  const T rm = pload(P.rho0_t, c.k - 1, g.nz), rp = pload(P.rho0_t, c.k + 1, g.nz);
  const T n0 = nu[(int64_t)c.i + (int64_t)g.nx * c.j + g.nxy * c.k];
  FaceVisc<T> f;
  f.xp = r0 * (T(0.5) * (n0 + gload(nu, g, c.i + 1, c.j, c.k, T(1))));
  f.xm = r0 * (T(0.5) * (gload(nu, g, c.i - 1, c.j, c.k, T(1)) + n0));
  f.yp = r0 * (T(0.5) * (n0 + gload(nu, g, c.i, c.j + 1, c.k, T(1))));
  f.ym = r0 * (T(0.5) * (gload(nu, g, c.i, c.j - 1, c.k, T(1)) + n0));
  f.zp = T(0.5) * (r0 + rp) * (T(0.5) * (n0 + gload(nu, g, c.i, c.j, c.k + 1, T(1))));
  f.zm = T(0.5) * (rm + r0) * (T(0.5) * (gload(nu, g, c.i, c.j, c.k - 1, T(1)) + n0));
  return f;
}

// div(rho0 nu / Pr grad s), compact face differences.
template <typename T>
__device__ __forceinline__ T diffuse(const Grid &g, const Dyn<T> &d, const FaceVisc<T> &f, T inv_pr,
                                     const T *__restrict__ s, const Cell &c) {
  const T s0 = gload(s, g, c.i, c.j, c.k, T(1));
  const T gx = (f.xp * inv_pr * ((gload(s, g, c.i + 1, c.j, c.k, T(1)) - s0) * d.inv_dx) -
                f.xm * inv_pr * ((s0 - gload(s, g, c.i - 1, c.j, c.k, T(1))) * d.inv_dx)) *
               d.inv_dx;
  const T gy = (f.yp * inv_pr * ((gload(s, g, c.i, c.j + 1, c.k, T(1)) - s0) * d.inv_dy) -
                f.ym * inv_pr * ((s0 - gload(s, g, c.i, c.j - 1, c.k, T(1))) * d.inv_dy)) *
               d.inv_dy;
  const T gz = (f.zp * inv_pr * ((gload(s, g, c.i, c.j, c.k + 1, T(1)) - s0) * d.inv_dz) -
                f.zm * inv_pr * ((s0 - gload(s, g, c.i, c.j, c.k - 1, T(1))) * d.inv_dz)) *
               d.inv_dz;
  return gx + gy + gz;
}

// Phi^{k+1} = Phi^{n+1/2} + dt/rho0 [ -div(U^k Phi_mid) + div(rho0 nu/Pr grad Phi_mid)
//            + rho0 w_sub dPhi_mid/dz + radiative heating (theta_l) + surface flux ]
template <typename T, bool WENO>
__global__ __launch_bounds__(kBlock) void scalar_kernel(
    Grid g, Dyn<T> d, Profiles<T> P, const T *__restrict__ u, const T *__restrict__ v,
    const T *__restrict__ w, const T *__restrict__ thm, const T *__restrict__ qtm,
    const T *__restrict__ thh, const T *__restrict__ qth, const T *__restrict__ nu,
    const T *__restrict__ rad, T *__restrict__ tho, T *__restrict__ qto) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const Cell c = cell_of(g, q);
  const FaceFlux<T> mf = face_mass(g, P, u, v, w, c);
  const FaceVisc<T> fv = face_visc(g, P, nu, c);
  const T r0 = P.rho0_t[c.k];
  const T sub = r0 * P.wsub_t[c.k];
  const T scale = d.dt / r0;
  {
    T tend = advect<T, WENO>(g, d, mf, thm, T(1), c) + diffuse(g, d, fv, d.inv_pr, thm, c);
    tend += rad[q];
    tend += sub * ((gload(thm, g, c.i, c.j, c.k + 1, T(1)) - gload(thm, g, c.i, c.j, c.k - 1, T(1))) * d.inv_2dz);
    if (c.k == 0) tend += d.sfc_thl * d.inv_dz;
    tho[q] = thh[q] + scale * tend;
  }
  {
    T tend = advect<T, WENO>(g, d, mf, qtm, T(1), c) + diffuse(g, d, fv, d.inv_sc, qtm, c);
    tend += sub * ((gload(qtm, g, c.i, c.j, c.k + 1, T(1)) - gload(qtm, g, c.i, c.j, c.k - 1, T(1))) * d.inv_2dz);
    if (c.k == 0) tend += d.sfc_qt * d.inv_dz;
    qto[q] = qth[q] + scale * tend;
  }
}

// ------------------------------------------------------ momentum update

// SGS momentum flux of component cmp through the face between cell a and
// cell b = a + e_ax: rho0_f nu_f [ (u_cmp(b) - u_cmp(a))/Delta_ax
//   + (d u_ax/d x_cmp (a) + d u_ax/d x_cmp (b)) / 2 ].
template <typename T, bool FS>
__device__ __forceinline__ T sgs_face(const Grid &g, const Dyn<T> &d, const T *const vel[3], T rnu,
                                      int ax, int cmp, int ia, int ja, int ka) {
  const int di = ax == 0, dj = ax == 1, dk = ax == 2;
  const T inv = ax == 0 ? d.inv_dx : (ax == 1 ? d.inv_dy : d.inv_dz);
  const T normal = (gload(vel[cmp], g, ia + di, ja + dj, ka + dk, vpar<T, FS>(cmp)) -
                    gload(vel[cmp], g, ia, ja, ka, vpar<T, FS>(cmp))) *
                   inv;
  const T trans = T(0.5) * (dcentral<T, FS>(vel[ax], g, d, ax, cmp, ia, ja, ka) +
                            dcentral<T, FS>(vel[ax], g, d, ax, cmp, ia + di, ja + dj, ka + dk));
  return rnu * (normal + trans);
}

// U_hat = U^n + dt [ -rho0 grad_c(alpha0 p^k) + R^{n+1/2} ] with
// R = -div(U_h (x) u_h) + div(rho0 sigma) + rho0 b e_z - f e_z x (U_h - rho0 u_g)
//     - beta(z) (U_h - rho0 (u_g, v_g, 0)); stored as u_hat = U_hat / rho0.
template <typename T, bool WENO, bool FS>
__global__ __launch_bounds__(kBlock) void momentum_kernel(
    Grid g, Dyn<T> d, Profiles<T> P, const T *__restrict__ uh, const T *__restrict__ vh,
    const T *__restrict__ wh, const T *__restrict__ un, const T *__restrict__ vn,
    const T *__restrict__ wn, const T *__restrict__ p, const T *__restrict__ b,
    const T *__restrict__ nu, T *__restrict__ uo, T *__restrict__ vo, T *__restrict__ wo) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const Cell c = cell_of(g, q);
  const T *const vel[3] = {uh, vh, wh};
  const FaceFlux<T> mf = face_mass(g, P, uh, vh, wh, c);
  const FaceVisc<T> fv = face_visc(g, P, nu, c);
  const T r0 = P.rho0_t[c.k];
  const T beta = P.beta_t[c.k];
  // pressure gradient of psi = alpha0 p' (even mirror)
  auto psi = [&](int i, int j, int k) {
    return pload(P.alpha0_t, k, g.nz) * gload(p, g, i, j, k, T(1));
  };
  const T gpx = (psi(c.i + 1, c.j, c.k) - psi(c.i - 1, c.j, c.k)) * d.inv_2dx;
  const T gpy = (psi(c.i, c.j + 1, c.k) - psi(c.i, c.j - 1, c.k)) * d.inv_2dy;
  const T gpz = (psi(c.i, c.j, c.k + 1) - psi(c.i, c.j, c.k - 1)) * d.inv_2dz;
  const T gp[3] = {gpx, gpy, gpz};
  const T Uh[3] = {r0 * uh[q], r0 * vh[q], r0 * wh[q]};
  const T Un[3] = {r0 * un[q], r0 * vn[q], r0 * wn[q]};
  const T geo[3] = {d.ug, d.vg, T(0)};
  T *const out[3] = {uo, vo, wo};
  const T rnu_m[3] = {fv.xm, fv.ym, fv.zm};
  const T rnu_p[3] = {fv.xp, fv.yp, fv.zp};
  const T invd[3] = {d.inv_dx, d.inv_dy, d.inv_dz};
#pragma unroll
  for (int cmp = 0; cmp < 3; ++cmp) {
    T R = advect<T, WENO>(g, d, mf, vel[cmp], vpar<T, FS>(cmp), c);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int di = ax == 0, dj = ax == 1, dk = ax == 2;
      const T fp = sgs_face<T, FS>(g, d, vel, rnu_p[ax], ax, cmp, c.i, c.j, c.k);
      const T fm = sgs_face<T, FS>(g, d, vel, rnu_m[ax], ax, cmp, c.i - di, c.j - dj, c.k - dk);
      R += (fp - fm) * invd[ax];
    }
    if (cmp == 2) R += r0 * b[q];
    if (cmp == 0) R += d.fcor * (Uh[1] - r0 * d.vg);
    if (cmp == 1) R -= d.fcor * (Uh[0] - r0 * d.ug);
    R -= beta * (Uh[cmp] - r0 * geo[cmp]);
    const T Uhat = Un[cmp] + d.dt * (-r0 * gp[cmp] + R);
    out[cmp][q] = Uhat / r0;
  }
}

}  // namespace

template <typename T>
void launch_sgs_nu(const Grid &g, const Dyn<T> &d, const T *u, const T *v, const T *w, const T *b,
                   T *nu, hipStream_t s) {
  if (d.uv_par > T(0))
    sgs_nu_kernel<T, true><<<blocks_for(g.n), kBlock, 0, s>>>(g, d, u, v, w, b, nu);
  else
    sgs_nu_kernel<T, false><<<blocks_for(g.n), kBlock, 0, s>>>(g, d, u, v, w, b, nu);
}

template <typename T>
void launch_scalar_update(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                          const T *v, const T *w, const T *thl_mid, const T *qt_mid,
                          const T *thl_half, const T *qt_half, const T *nu, const T *rad,
                          T *thl_out, T *qt_out, hipStream_t s) {
  if (d.advection == LES_WENO3)
    scalar_kernel<T, true><<<blocks_for(g.n), kBlock, 0, s>>>(
        g, d, P, u, v, w, thl_mid, qt_mid, thl_half, qt_half, nu, rad, thl_out, qt_out);
  else
    scalar_kernel<T, false><<<blocks_for(g.n), kBlock, 0, s>>>(
        g, d, P, u, v, w, thl_mid, qt_mid, thl_half, qt_half, nu, rad, thl_out, qt_out);
}

template <typename T>
void launch_momentum(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *uh,
                     const T *vh, const T *wh, const T *un, const T *vn, const T *wn, const T *p,
                     const T *b, const T *nu, T *uo, T *vo, T *wo, hipStream_t s) {
#define LES_MOM(WENO, FS)                                                                \
  momentum_kernel<T, WENO, FS><<<blocks_for(g.n), kBlock, 0, s>>>(g, d, P, uh, vh, wh, un, vn, \
                                                                  wn, p, b, nu, uo, vo, wo)
  const bool weno = d.advection == LES_WENO3, fs = d.uv_par > T(0);
  if (weno && fs) LES_MOM(true, true);
  else if (weno) LES_MOM(true, false);
  else if (fs) LES_MOM(false, true);
  else LES_MOM(false, false);
#undef LES_MOM
}

#define LES_INST(T)                                                                              \
  template void launch_sgs_nu<T>(const Grid &, const Dyn<T> &, const T *, const T *, const T *,  \
                                 const T *, T *, hipStream_t);                                   \
  template void launch_scalar_update<T>(const Grid &, const Dyn<T> &, const Profiles<T> &,       \
                                        const T *, const T *, const T *, const T *, const T *,   \
                                        const T *, const T *, const T *, const T *, T *, T *,    \
                                        hipStream_t);                                            \
  template void launch_momentum<T>(const Grid &, const Dyn<T> &, const Profiles<T> &, const T *, \
                                   const T *, const T *, const T *, const T *, const T *,        \
                                   const T *, const T *, const T *, T *, T *, T *, hipStream_t);
LES_INST(float)
LES_INST(double)
#undef LES_INST

}  // namespace lesmi
