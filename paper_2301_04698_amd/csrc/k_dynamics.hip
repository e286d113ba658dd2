// Subgrid viscosity (paper Sec. 2.3), scalar predictor (Sec. 2.4, scalar
// prediction equation) and momentum predictor (Sec. 2.4, momentum
// prediction equation) on the collocated grid.  Column-marching kernels
// (one lane per column, a chunk of levels per wave); the stencil
// neighbourhoods are served by the L1/L2 caches.
#include <type_traits>

#include "les.h"
#include "les_column.h"
#include "les_tile.h"

namespace lesmi {

namespace {

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
// the cell offset (oi, oj, ok) from the wave's cell (a ghost level near
// the walls).
template <typename T, bool FS, class L>
__device__ __forceinline__ T dcentral(const T *__restrict__ f, const L &at, const Dyn<T> &d, int a,
                                      int ax, int oi, int oj, int ok) {
  const int di = ax == 0, dj = ax == 1, dk = ax == 2;
  const T inv2 = ax == 0 ? d.inv_2dx : (ax == 1 ? d.inv_2dy : d.inv_2dz);
  const T par = vpar<T, FS>(a);
  return (at(f, oi + di, oj + dj, ok + dk, par) - at(f, oi - di, oj - dj, ok - dk, par)) * inv2;
}

// ---------------------------------------------------------------- SGS nu

// nu_t = (c_s Delta)^2 f_B S with S = sqrt(2 S_ij S_ij) and the buoyancy
// factor f_B = sqrt(clamp(1 - N^2/(Pr S^2), 0, 1)), N^2 = db/dz (central);
// or the uniform viscosity of the validation cases (Sec. 3) when set.
// Tiled z march (les_tile.h): the x and y differences of u, v, w from their
// LDS planes, the z differences (and N^2) from the column's values below
// and above carried in registers.
template <typename T, bool FS>
__global__ __launch_bounds__(kTileThreads) void sgs_nu_kernel(Grid g, TileMap m, Dyn<T> d,
                                                              const T *__restrict__ u,
                                                              const T *__restrict__ v,
                                                              const T *__restrict__ w,
                                                              const T *__restrict__ b,
                                                              T *__restrict__ nu) {
  __shared__ TilePlane<T, 1, 1> pl[2][3];  // u, v, w at the level, two slots
  const Tile tl = tile_of(g, m);
  if (!tl.valid) return;
  const TileCol c = tile_col(g, tl);
  if (d.nu_const > T(0)) {
    for (int k = tl.k0; k < tl.k1; ++k)
      if (c.active) nu[(int64_t)k * g.nxy + c.off] = d.nu_const;
    return;
  }
  const RingCells<1, 1> rc = ring_cells<1, 1>(g, tl);
  constexpr int PER = RingCells<1, 1>::PER;
  const T *const fld[4] = {u, v, w, b};
  const T fpar[4] = {vpar<T, FS>(0), vpar<T, FS>(1), vpar<T, FS>(2), T(1)};
  // Loads run ahead of the march in register FIFOs of depth D indexed by
  // the level's place i = k - k0 in the chunk: the ring cells of level k in
  // slot i % D (fetched D levels ahead), the column's u, v, w, b at level k
  // in slot (i + 1) % D (levels k - 1 .. k + D - 2 held; fetched D - 1
  // levels ahead, up to level k1, the last one the march reads).
  constexpr int D = kTileDepth;
  T hq[D][3][PER], zq[D][4];
  auto fetch_ring = [&](T(&h)[3][PER], int kk) __attribute__((always_inline)) {
    if (kk < tl.k1) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < PER; ++q)
          if (rc.dst[q] >= 0) h[a][q] = fld[a][(int64_t)kk * g.nxy + rc.src[q]];
    }
  };
  auto fetch_col = [&](T(&z)[4], int kk) __attribute__((always_inline)) {
    kk = min(kk, tl.k1);
#pragma unroll
    for (int f = 0; f < 4; ++f) z[f] = col_value(g, fld[f], c.off, kk, fpar[f]);
  };
#pragma unroll
  for (int s = 0; s < D; ++s) {
    fetch_ring(hq[s], tl.k0 + s);
    fetch_col(zq[s], tl.k0 - 1 + s);
  }
  const int x = c.lx + 1, y = c.ly + 1;
  // level k = k0 + i, i = PH (mod 4)
  auto level = [&](auto ph, int k) __attribute__((always_inline)) {
    constexpr int PH = decltype(ph)::value;
    T(&zm)[4] = zq[PH];
    T(&z0)[4] = zq[(PH + 1) % D];
    T(&zp)[4] = zq[(PH + 2) % D];
    TilePlane<T, 1, 1> *P = pl[PH & 1];
    // this slot was last read two levels ago, before the last barrier
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P[a].v[y][x] = z0[a];
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (rc.dst[q] >= 0) (&P[a].v[0][0])[rc.dst[q]] = hq[PH][a][q];
    }
    fetch_ring(hq[PH], k + D);
    __syncthreads();
    T G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      G[a][0] = (P[a].v[y][x + 1] - P[a].v[y][x - 1]) * d.inv_2dx;
      G[a][1] = (P[a].v[y + 1][x] - P[a].v[y - 1][x]) * d.inv_2dy;
      G[a][2] = (zp[a] - zm[a]) * d.inv_2dz;
    }
    // S^2 = 2 S_ij S_ij: the diagonal terms plus the three distinct
    // off-diagonal pairs (S_ij = S_ji)
    const T o01 = G[0][1] + G[1][0], o02 = G[0][2] + G[2][0], o12 = G[1][2] + G[2][1];
    const T s2 = T(2) * (G[0][0] * G[0][0] + G[1][1] * G[1][1] + G[2][2] * G[2][2]) +
                 (o01 * o01 + o02 * o02 + o12 * o12);
    const T n2 = (zp[3] - zm[3]) * d.inv_2dz;
    // S^2 f_B^2 = S^2 clamp(1 - N^2/(Pr S^2), 0, 1) = clamp(S^2 - N^2/Pr, 0, S^2)
    T e2 = s2 - n2 * d.inv_pr;
    e2 = e2 < T(0) ? T(0) : (e2 > s2 ? s2 : e2);
    const T val = d.smag_l2 * sqrt(e2);
    if (c.active) nu[(int64_t)k * g.nxy + c.off] = val;
    fetch_col(zq[PH], k - 1 + D);  // the slot of level k - 1, used for the last time
  };
  for (int k = tl.k0; march_trip(level, k, tl.k1, std::make_integer_sequence<int, D>{}); k += D) {
  }
}

// ------------------------------------------------------- scalar update

// Face mass fluxes of the six faces of a cell: average of rho0 u of the
// two cells sharing the face (zero on the walls by the odd mirror of w).
template <typename T>
struct FaceFlux {
  T xm, xp, ym, yp, zm, zp;
};

template <typename T, class L>
__device__ __forceinline__ FaceFlux<T> face_mass(const L &at, const Profiles<T> &P,
                                                 const T *__restrict__ u, const T *__restrict__ v,
                                                 const T *__restrict__ w) {
  const T r0 = at.prof(P.rho0_t, 0);
  const T rm = at.prof(P.rho0_t, -1), rp = at.prof(P.rho0_t, 1);
  const T uc = r0 * at(u, 0, 0, 0, T(-1));
  const T vc = r0 * at(v, 0, 0, 0, T(-1));
  const T wc = r0 * at(w, 0, 0, 0, T(-1));
  FaceFlux<T> f;
  f.xp = T(0.5) * (uc + r0 * at(u, 1, 0, 0, T(-1)));
  f.xm = T(0.5) * (r0 * at(u, -1, 0, 0, T(-1)) + uc);
  f.yp = T(0.5) * (vc + r0 * at(v, 0, 1, 0, T(-1)));
  f.ym = T(0.5) * (r0 * at(v, 0, -1, 0, T(-1)) + vc);
  f.zp = T(0.5) * (wc + rp * at(w, 0, 0, 1, T(-1)));
  f.zm = T(0.5) * (rm * at(w, 0, 0, -1, T(-1)) + wc);
  return f;
}

// Flux-form advective tendency -div(U s) of a field s with parity par.
// The flux through the bottom face is the one the level below computed for
// its top face when `have` (the same operands in the same order, so the
// same value): zin (HAVE); the top face's flux goes to zout for the level
// above.
template <typename T, bool WENO, bool HAVE, class L>
__device__ __forceinline__ T advect(const L &at, const Dyn<T> &d, const FaceFlux<T> &f,
                                    const T *__restrict__ s, T par, T zin, T &zout) {
  T sx[5], sy[5], sz[5];
#pragma unroll
  for (int o = -2; o <= 2; ++o) {
    sx[o + 2] = at(s, o, 0, 0, par);
    sy[o + 2] = at(s, 0, o, 0, par);
    sz[o + 2] = at(s, 0, 0, o, par);
  }
  const T fxp = face_flux<T, WENO>(f.xp, sx[1], sx[2], sx[3], sx[4]);
  const T fxm = face_flux<T, WENO>(f.xm, sx[0], sx[1], sx[2], sx[3]);
  const T fyp = face_flux<T, WENO>(f.yp, sy[1], sy[2], sy[3], sy[4]);
  const T fym = face_flux<T, WENO>(f.ym, sy[0], sy[1], sy[2], sy[3]);
  const T fzp = face_flux<T, WENO>(f.zp, sz[1], sz[2], sz[3], sz[4]);
  T fzm;
  if constexpr (HAVE)
    fzm = zin;
  else
    fzm = face_flux<T, WENO>(f.zm, sz[0], sz[1], sz[2], sz[3]);
  zout = fzp;
  return -((fxp - fxm) * d.inv_dx + (fyp - fym) * d.inv_dy + (fzp - fzm) * d.inv_dz);
}

// Viscosity and rho0 on the six faces (means of the two adjacent cells).
template <typename T>
struct FaceVisc {
  T xm, xp, ym, yp, zm, zp;  // rho0_f * nu_f
};

template <typename T, class L>
__device__ __forceinline__ FaceVisc<T> face_visc(const L &at, const Profiles<T> &P,
                                                 const T *__restrict__ nu) {
  const T r0 = at.prof(P.rho0_t, 0);
  const T rm = at.prof(P.rho0_t, -1), rp = at.prof(P.rho0_t, 1);
  const T n0 = at(nu, 0, 0, 0, T(1));
  FaceVisc<T> f;
  f.xp = r0 * (T(0.5) * (n0 + at(nu, 1, 0, 0, T(1))));
  f.xm = r0 * (T(0.5) * (at(nu, -1, 0, 0, T(1)) + n0));
  f.yp = r0 * (T(0.5) * (n0 + at(nu, 0, 1, 0, T(1))));
  f.ym = r0 * (T(0.5) * (at(nu, 0, -1, 0, T(1)) + n0));
  f.zp = T(0.5) * (r0 + rp) * (T(0.5) * (n0 + at(nu, 0, 0, 1, T(1))));
  f.zm = T(0.5) * (rm + r0) * (T(0.5) * (at(nu, 0, 0, -1, T(1)) + n0));
  return f;
}

// div(rho0 nu / Pr grad s), compact face differences; the bottom face's
// flux carried from the level below as in advect.
template <typename T, bool HAVE, class L>
__device__ __forceinline__ T diffuse(const L &at, const Dyn<T> &d, const FaceVisc<T> &f, T inv_pr,
                                     const T *__restrict__ s, T zin, T &zout) {
  const T s0 = at(s, 0, 0, 0, T(1));
  const T gx = (f.xp * inv_pr * ((at(s, 1, 0, 0, T(1)) - s0) * d.inv_dx) -
                f.xm * inv_pr * ((s0 - at(s, -1, 0, 0, T(1))) * d.inv_dx)) *
               d.inv_dx;
  const T gy = (f.yp * inv_pr * ((at(s, 0, 1, 0, T(1)) - s0) * d.inv_dy) -
                f.ym * inv_pr * ((s0 - at(s, 0, -1, 0, T(1))) * d.inv_dy)) *
               d.inv_dy;
  const T fzp = f.zp * inv_pr * ((at(s, 0, 0, 1, T(1)) - s0) * d.inv_dz);
  T fzm;
  if constexpr (HAVE)
    fzm = zin;
  else
    fzm = f.zm * inv_pr * ((s0 - at(s, 0, 0, -1, T(1))) * d.inv_dz);
  zout = fzp;
  const T gz = (fzp - fzm) * d.inv_dz;
  return gx + gy + gz;
}

// Bottom-face fluxes a level hands to the level above in a z march.
template <typename T, int N>
struct ZCarry {
  T f[N];
};

// Phi^{k+1} = Phi^{n+1/2} + dt/rho0 [ -div(U^k Phi_mid) + div(rho0 nu/Pr grad Phi_mid)
//            + rho0 w_sub dPhi_mid/dz + radiative heating (theta_l) + surface flux ]
template <typename T, bool WENO, bool EDGE, bool HAVE>
__device__ __forceinline__ void scalar_level(
    const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const ColPts<T> &pts, int k,
    bool active, const T *__restrict__ u, const T *__restrict__ v, const T *__restrict__ w,
    const T *__restrict__ thm, const T *__restrict__ qtm, const T *__restrict__ thh,
    const T *__restrict__ qth, const T *__restrict__ nu, const T *__restrict__ rad,
    T *__restrict__ tho, T *__restrict__ qto, ZCarry<T, 4> &zc) {
  const Lvl<T, EDGE> at(g, pts, k);
  const FaceFlux<T> mf = face_mass(at, P, u, v, w);
  const FaceVisc<T> fv = face_visc(at, P, nu);
  const T r0 = at.prof(P.rho0_t, 0);
  const T sub = r0 * at.prof(P.wsub_t, 0);
  const T scale = d.dt / r0;
  T th_new, qt_new;
  ZCarry<T, 4> out;
  {
    T tend = advect<T, WENO, HAVE>(at, d, mf, thm, T(1), zc.f[0], out.f[0]) +
             diffuse<T, HAVE>(at, d, fv, d.inv_pr, thm, zc.f[1], out.f[1]);
    tend += at(rad, 0, 0, 0, T(1));
    tend += sub * ((at(thm, 0, 0, 1, T(1)) - at(thm, 0, 0, -1, T(1))) * d.inv_2dz);
    if (k == 0) tend += d.sfc_thl * d.inv_dz;
    th_new = at(thh, 0, 0, 0, T(1)) + scale * tend;
  }
  {
    T tend = advect<T, WENO, HAVE>(at, d, mf, qtm, T(1), zc.f[2], out.f[2]) +
             diffuse<T, HAVE>(at, d, fv, d.inv_sc, qtm, zc.f[3], out.f[3]);
    tend += sub * ((at(qtm, 0, 0, 1, T(1)) - at(qtm, 0, 0, -1, T(1))) * d.inv_2dz);
    if (k == 0) tend += d.sfc_qt * d.inv_dz;
    qt_new = at(qth, 0, 0, 0, T(1)) + scale * tend;
  }
  // Stores after all loads (the two scalars share the face fluxes' loads).
  at.store(tho, th_new, active);
  at.store(qto, qt_new, active);
  zc = out;
}

template <typename T, bool WENO>
__global__ __launch_bounds__(kBlock) void scalar_kernel(
    Grid g, ColMap m, Dyn<T> d, Profiles<T> P, const T *__restrict__ u, const T *__restrict__ v,
    const T *__restrict__ w, const T *__restrict__ thm, const T *__restrict__ qtm,
    const T *__restrict__ thh, const T *__restrict__ qth, const T *__restrict__ nu,
    const T *__restrict__ rad, T *__restrict__ tho, T *__restrict__ qto) {
  const ColWave c = col_wave(g, m);
  if (!c.valid) return;
  const ColPts<T> pts = col_pts<T>(g, c.i, c.j);
  // the chunk's first level computes its bottom faces; the others take
  // them from the level below
  ZCarry<T, 4> zc = {};
  scalar_level<T, WENO, true, false>(g, d, P, pts, c.k0, c.active, u, v, w, thm, qtm, thh, qth,
                                     nu, rad, tho, qto, zc);
  for (int k = c.k0 + 1; k < c.k1; ++k) {
    if (k >= 2 && k + 2 < g.nz)
      scalar_level<T, WENO, false, true>(g, d, P, pts, k, c.active, u, v, w, thm, qtm, thh, qth,
                                         nu, rad, tho, qto, zc);
    else
      scalar_level<T, WENO, true, true>(g, d, P, pts, k, c.active, u, v, w, thm, qtm, thh, qth, nu,
                                        rad, tho, qto, zc);
  }
}

// ------------------------------------------------------ momentum update

// SGS momentum flux of component cmp through the face between the cell
// at offset o = (oi, oj, ok) and the one at o + e_ax:
//   rho0_f nu_f [ (u_cmp(o + e_ax) - u_cmp(o))/Delta_ax
//                 + (d u_ax/d x_cmp (o) + d u_ax/d x_cmp (o + e_ax)) / 2 ].
template <typename T, bool FS, class L>
__device__ __forceinline__ T sgs_face(const L &at, const Dyn<T> &d, const T *const vel[3], T rnu,
                                      int ax, int cmp, int oi, int oj, int ok) {
  const int di = ax == 0, dj = ax == 1, dk = ax == 2;
  const T inv = ax == 0 ? d.inv_dx : (ax == 1 ? d.inv_dy : d.inv_dz);
  const T normal = (at(vel[cmp], oi + di, oj + dj, ok + dk, vpar<T, FS>(cmp)) -
                    at(vel[cmp], oi, oj, ok, vpar<T, FS>(cmp))) *
                   inv;
  const T trans = T(0.5) * (dcentral<T, FS>(vel[ax], at, d, ax, cmp, oi, oj, ok) +
                            dcentral<T, FS>(vel[ax], at, d, ax, cmp, oi + di, oj + dj, ok + dk));
  return rnu * (normal + trans);
}

// U_hat = U^n + dt [ -rho0 grad_c(alpha0 p^k) + R^{n+1/2} ] with
// R = -div(U_h (x) u_h) + div(rho0 sigma) + rho0 b e_z - f e_z x (U_h - rho0 u_g)
//     - beta(z) (U_h - rho0 (u_g, v_g, 0)); stored as u_hat = U_hat / rho0.
template <typename T, bool WENO, bool FS, bool EDGE, bool HAVE>
__device__ __forceinline__ void momentum_level(
    const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const ColPts<T> &pts, int k,
    bool active, const T *__restrict__ uh, const T *__restrict__ vh, const T *__restrict__ wh,
    const T *__restrict__ un, const T *__restrict__ vn, const T *__restrict__ wn,
    const T *__restrict__ p, const T *__restrict__ b, const T *__restrict__ nu,
    T *__restrict__ uo, T *__restrict__ vo, T *__restrict__ wo, ZCarry<T, 6> &zc) {
  const Lvl<T, EDGE> at(g, pts, k);
  const T *const vel[3] = {uh, vh, wh};
  const FaceFlux<T> mf = face_mass(at, P, uh, vh, wh);
  const FaceVisc<T> fv = face_visc(at, P, nu);
  const T r0 = at.prof(P.rho0_t, 0);
  const T beta = at.prof(P.beta_t, 0);
  // pressure gradient of psi = alpha0 p' (even mirror)
  const T a0 = at.prof(P.alpha0_t, 0);
  const T gpx = (a0 * at(p, 1, 0, 0, T(1)) - a0 * at(p, -1, 0, 0, T(1))) * d.inv_2dx;
  const T gpy = (a0 * at(p, 0, 1, 0, T(1)) - a0 * at(p, 0, -1, 0, T(1))) * d.inv_2dy;
  // plus the gradient of the horizontally uniform part of p', kept as an
  // FP64 profile and rounded once
  const T gpz = (at.prof(P.alpha0_t, 1) * at(p, 0, 0, 1, T(1)) -
                 at.prof(P.alpha0_t, -1) * at(p, 0, 0, -1, T(1))) *
                    d.inv_2dz +
                at.prof(P.pgz_t, 0);
  const T gp[3] = {gpx, gpy, gpz};
  const T Uh[3] = {r0 * at(uh, 0, 0, 0, T(1)), r0 * at(vh, 0, 0, 0, T(1)),
                   r0 * at(wh, 0, 0, 0, T(1))};
  const T Un[3] = {r0 * at(un, 0, 0, 0, T(1)), r0 * at(vn, 0, 0, 0, T(1)),
                   r0 * at(wn, 0, 0, 0, T(1))};
  const T geo[3] = {d.ug, d.vg, T(0)};
  T *const outf[3] = {uo, vo, wo};
  const T rnu_m[3] = {fv.xm, fv.ym, fv.zm};
  const T rnu_p[3] = {fv.xp, fv.yp, fv.zp};
  const T invd[3] = {d.inv_dx, d.inv_dy, d.inv_dz};
  const T bq = at(b, 0, 0, 0, T(1));
  T res[3];
  ZCarry<T, 6> out;  // per component: advective, then SGS flux of the top face
#pragma unroll
  for (int cmp = 0; cmp < 3; ++cmp) {
    T R = advect<T, WENO, HAVE>(at, d, mf, vel[cmp], vpar<T, FS>(cmp), zc.f[cmp], out.f[cmp]);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int di = ax == 0, dj = ax == 1, dk = ax == 2;
      const T fp = sgs_face<T, FS>(at, d, vel, rnu_p[ax], ax, cmp, 0, 0, 0);
      // the z face below: the level below's top face when it was computed
      T fm;
      if (HAVE && ax == 2)
        fm = zc.f[3 + cmp];
      else
        fm = sgs_face<T, FS>(at, d, vel, rnu_m[ax], ax, cmp, -di, -dj, -dk);
      if (ax == 2) out.f[3 + cmp] = fp;
      R += (fp - fm) * invd[ax];
    }
    if (cmp == 2) R += r0 * bq;
    if (cmp == 0) R += d.fcor * (Uh[1] - r0 * d.vg);
    if (cmp == 1) R -= d.fcor * (Uh[0] - r0 * d.ug);
    R -= beta * (Uh[cmp] - r0 * geo[cmp]);
    const T Uhat = Un[cmp] + d.dt * (-r0 * gp[cmp] + R);
    res[cmp] = Uhat / r0;
  }
  // Stores after all loads: the loads of the three components share their
  // common points and differences.
#pragma unroll
  for (int cmp = 0; cmp < 3; ++cmp) at.store(outf[cmp], res[cmp], active);
  zc = out;
}

template <typename T, bool WENO, bool FS>
__global__ __launch_bounds__(kBlock) void momentum_kernel(
    Grid g, ColMap m, Dyn<T> d, Profiles<T> P, const T *__restrict__ uh, const T *__restrict__ vh,
    const T *__restrict__ wh, const T *__restrict__ un, const T *__restrict__ vn,
    const T *__restrict__ wn, const T *__restrict__ p, const T *__restrict__ b,
    const T *__restrict__ nu, T *__restrict__ uo, T *__restrict__ vo, T *__restrict__ wo) {
  const ColWave c = col_wave(g, m);
  if (!c.valid) return;
  const ColPts<T> pts = col_pts<T>(g, c.i, c.j);
  // the chunk's first level computes its bottom faces; the others take
  // them from the level below
  ZCarry<T, 6> zc = {};
  momentum_level<T, WENO, FS, true, false>(g, d, P, pts, c.k0, c.active, uh, vh, wh, un, vn, wn, p,
                                           b, nu, uo, vo, wo, zc);
  for (int k = c.k0 + 1; k < c.k1; ++k) {
    if (k >= 2 && k + 2 < g.nz)
      momentum_level<T, WENO, FS, false, true>(g, d, P, pts, k, c.active, uh, vh, wh, un, vn, wn,
                                               p, b, nu, uo, vo, wo, zc);
    else
      momentum_level<T, WENO, FS, true, true>(g, d, P, pts, k, c.active, uh, vh, wh, un, vn, wn, p,
                                              b, nu, uo, vo, wo, zc);
  }
}

}  // namespace

template <typename T>
void launch_sgs_nu(const Grid &g, const Dyn<T> &d, const T *u, const T *v, const T *w, const T *b,
                   T *nu, hipStream_t s) {
  const TileMap m = tile_map(g);
  if (d.uv_par > T(0))
    sgs_nu_kernel<T, true><<<m.blocks, kTileThreads, 0, s>>>(g, m, d, u, v, w, b, nu);
  else
    sgs_nu_kernel<T, false><<<m.blocks, kTileThreads, 0, s>>>(g, m, d, u, v, w, b, nu);
}

template <typename T>
void launch_scalar_update(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                          const T *v, const T *w, const T *thl_mid, const T *qt_mid,
                          const T *thl_half, const T *qt_half, const T *nu, const T *rad,
                          T *thl_out, T *qt_out, hipStream_t s) {
  const ColMap m = col_map(g);
  if (d.advection == LES_WENO3)
    scalar_kernel<T, true><<<m.blocks, kBlock, 0, s>>>(
        g, m, d, P, u, v, w, thl_mid, qt_mid, thl_half, qt_half, nu, rad, thl_out, qt_out);
  else
    scalar_kernel<T, false><<<m.blocks, kBlock, 0, s>>>(
        g, m, d, P, u, v, w, thl_mid, qt_mid, thl_half, qt_half, nu, rad, thl_out, qt_out);
}

template <typename T>
void launch_momentum(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *uh,
                     const T *vh, const T *wh, const T *un, const T *vn, const T *wn, const T *p,
                     const T *b, const T *nu, T *uo, T *vo, T *wo, hipStream_t s) {
  const ColMap m = col_map(g);
#define LES_MOM(WENO, FS)                                                                     \
  momentum_kernel<T, WENO, FS><<<m.blocks, kBlock, 0, s>>>(g, m, d, P, uh, vh, wh, un, vn, wn, \
                                                           p, b, nu, uo, vo, wo)
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
