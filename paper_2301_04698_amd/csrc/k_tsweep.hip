// Weighted-Jacobi / Chebyshev sweeps of the compact 7-point
// pressure-correction operator (paper Sec. 2.4 and App. A), one or two
// sweeps per launch.
//
// Point update, shared by every kernel so their results are bitwise equal:
//   r   = rhs - (N(phi) - D phi)     N: off-diagonal neighbour sum, FP64
//   J   = phi - omega_j r / D         (weighted Jacobi)
//   out = J, or Chebyshev: prev + omega_c (J - prev)
// formed in FP64 from the stored values with explicit FMAs (no other
// contraction) and rounded once to the storage type.  An FP32 update
// written as (N - rhs)/D - phi cancels catastrophically; its rounding error
// is the same from sweep to sweep and accumulates in the slow modes.
//
// One sweep: each thread owns one column of the tile and marches up z
// with the vertical neighbours in registers; x neighbours come from the
// adjacent lanes of the wavefront, y neighbours through the L1/L2 caches.
// 16 bytes per cell (Chebyshev: phi, prev, rhs in, phi' out).  Grids at
// least 256 cells wide take 256-cell-wide tiles (four waves side by side):
// 256 x 2 while the four arrays fit the 256 MB Infinity Cache, 256 x 4
// beyond it, where the arrays read once per sweep (prev, rhs) and the
// output are streamed with non-temporal accesses so the caches keep the
// iterate's neighbour rows.  Narrower grids take 64 x 4 (or 64 x 16
// streamed, 64 x 1 for ny < 4) tiles.
//
// Two sweeps: a 64 x TY thread tile covers a 62 x (TY-2) core plus a
// one-cell ring.  Every thread computes the first sweep for its own column
// as above; the second sweep, on the core only, takes the first sweep's x/y
// neighbours from a ring of LDS planes and its z neighbours from the
// thread's own registers.  20 bytes per cell for both sweeps.
//
// Walls: the z neighbour of the bottom/top level is that level itself (even
// mirror); x and y are periodic.
#include "les_device.h"

namespace lesmi {

namespace {

struct SweepCoef {
  double ix2, iy2, iz2, diag, inv_diag, omega_j;
};

__device__ __forceinline__ double point_residual(const SweepCoef &k, double c0, double hx,
                                                 double hy, double hz, double rhs) {
#pragma clang fp contract(off)
  const double lap = fma(hx, k.ix2, fma(hy, k.iy2, fma(hz, k.iz2, -k.diag * c0)));
  return rhs - lap;
}

__device__ __forceinline__ double point_update(const SweepCoef &k, double c0, double res,
                                               bool cheb, double pv, double wc) {
#pragma clang fp contract(off)
  const double jac = fma(-k.omega_j * k.inv_diag, res, c0);
  return cheb ? fma(wc, jac - pv, pv) : jac;
}

__device__ __forceinline__ int pmod(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Logical tile of physical block b.  Workgroups go to the 8 XCDs
// round-robin (b mod 8); each XCD gets one contiguous range of tiles
// (x fastest, then y, then z chunk), so the y halos a tile reads were
// fetched into the same L2 by its neighbours.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int per = nblocks >> 3;  // nblocks is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

template <typename T>
struct SweepArgs {
  Grid g;
  SweepCoef k;
  int kc, tiles_x, tiles_y, tiles_z, ntiles;
  double wc0, wc1;   // Chebyshev weights of the launch's first and second sweep
  int first;         // the first sweep is the first of the solve (weight 1, no prev)
  const T *cur, *prev, *rhs;
  T *out_last, *out_prev;
  SolveCtl *ctl;
  double *partials;
  // one-sweep launches: a pending residual check (sweep dec_m >= 0) of an
  // earlier launch whose dec_np block partials block 0 reduces and decides
  const double *dec_partials;
  int dec_np, dec_m;
};

struct TileIdx {
  int tx, ty, k0, k1;
};

__device__ __forceinline__ TileIdx tile_of(int tile, int tiles_x, int tiles_y, int kc, int nz) {
  TileIdx t;
  t.tx = tile % tiles_x;
  const int rest = tile / tiles_x;
  t.ty = rest % tiles_y;
  t.k0 = (rest / tiles_y) * kc;
  t.k1 = min(nz, t.k0 + kc);
  return t;
}

// ---------------------------------------------------------------- 1 sweep

constexpr int kTY1 = 4;       // cache-resident arrays
constexpr int kTY1Big = 16;   // streamed arrays
// Grids at least kWideNx wide take tiles of kWX waves side by side along x
// (256-cell rows): longer contiguous runs per plane row and fewer halo
// planes per cell; kWideTY rows when cache-resident, kWideTYBig streamed.
constexpr int kWideNx = 256, kWX = 4, kWideTY = 2, kWideTYBig = 4;

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p, bool nt) {
  return nt ? __builtin_nontemporal_load(p) : *p;
}

// Value of v in the next (+1) or previous (-1) lane of the 64-wide
// wavefront by DPP wave shifts; a lane without a source keeps its own value
// (the caller replaces the end lanes).  A double moves as two 32-bit halves.
template <int DIR>
__device__ __forceinline__ float lane_shift(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, DIR > 0 ? 0x130 : 0x138, 0xF, 0xF, false));
}
template <int DIR>
__device__ __forceinline__ double lane_shift(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int ctrl = DIR > 0 ? 0x130 : 0x138;
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, ctrl, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, ctrl, 0xF, 0xF, false));
}

// z-march of one 64-cell row (one wave) of a tile over levels [k0, k1):
// one Chebyshev (or, CHEB = false, weighted-Jacobi) sweep of each cell,
// returning its FP64 residual sum when CHECK.  SHIFT: the x neighbours of a
// cell are the iterate values its neighbouring lanes already hold (DPP wave
// shifts) and only the row's end lanes load theirs, so each plane row is
// read once; otherwise they are loaded.  FULL: all 64 cells of the row lie
// inside the grid, so no lane is predicated off (a predicated store makes
// the compiler wait for that store before the next level); a ragged row's
// lanes beyond nx march on the row's last cell, for the shifts, but neither
// store nor count in the residual.
template <bool FULL, bool SHIFT, bool CHEB, bool CHECK, bool NT, typename T>
__device__ __forceinline__ double march_row(const SweepArgs<T> &a, const TileIdx &t, int lane,
                                            int i, int j) {
  const Grid &g = a.g;
  const bool valid = FULL || i < g.nx;
  const int ic = valid ? i : g.nx - 1;
  const int ip = ic + 1 == g.nx ? 0 : ic + 1, im = ic == 0 ? g.nx - 1 : ic - 1;
  const int jp = j + 1 == g.ny ? 0 : j + 1, jm = j == 0 ? g.ny - 1 : j - 1;
  const int64_t col = (int64_t)ic + (int64_t)g.nx * j;
  const int64_t oxp = ip - ic, oxm = im - ic;
  const int64_t oyp = (int64_t)(jp - j) * g.nx, oym = (int64_t)(jm - j) * g.nx;
  const bool load_xp = lane == 63 || ic + 1 >= g.nx, load_xm = lane == 0;
  double acc = 0.0;
  T below = a.cur[col + g.nxy * (t.k0 > 0 ? t.k0 - 1 : 0)];
  T c = a.cur[col + g.nxy * t.k0];
  for (int k = t.k0; k < t.k1; ++k) {
    const int64_t q = col + g.nxy * k;
    const T above = a.cur[q + (k + 1 < g.nz ? g.nxy : 0)];
    T xp, xm;
    if (SHIFT) {
      xp = lane_shift<1>(c);
      xm = lane_shift<-1>(c);
      if (load_xp) xp = a.cur[q + oxp];
      if (load_xm) xm = a.cur[q + oxm];
    } else {
      xp = a.cur[q + oxp];
      xm = a.cur[q + oxm];
    }
    const double hx = (double)xp + (double)xm;
    const double hy = (double)a.cur[q + oyp] + (double)a.cur[q + oym];
    const double hz = (double)above + (double)below;
    const double res =
        point_residual(a.k, (double)c, hx, hy, hz, (double)ld_stream(&a.rhs[q], NT));
    if (CHECK && valid) acc += res * res;
    const double pv = CHEB ? (double)ld_stream(&a.prev[q], NT) : 0.0;
    const T out = (T)point_update(a.k, (double)c, res, CHEB, pv, a.wc0);
    if (valid) {
      if (NT)
        __builtin_nontemporal_store(out, &a.out_last[q]);
      else
        a.out_last[q] = out;
    }
    below = c;
    c = above;
  }
  return acc;
}

// A 64 WX x TY tile: wave (wx, wy) owns the 64 cells of row ty TY + wy
// starting at x = tx 64 WX + 64 wx.  The first sweep of a solve (weight 1,
// no previous iterate) launches as CHEB = false.  Lane shifts only in
// blocks of several waves: one-wave blocks (two-dimensional grids, few waves
// per CU) measured faster with loaded x neighbours.
template <typename T, int WX, int TY, bool CHEB, bool CHECK, bool NT>
__global__ __launch_bounds__(64 * WX * TY) void sweep1_kernel(SweepArgs<T> a) {
  if (a.ctl->done) return;
  const Grid &g = a.g;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  double acc = 0.0;
  if (tile < a.ntiles) {
    const TileIdx t = tile_of(tile, a.tiles_x, a.tiles_y, a.kc, g.nz);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int x0 = t.tx * 64 * WX + (wave % WX) * 64;
    const int i = x0 + lane;
    const int j = t.ty * TY + wave / WX;
    constexpr bool kShift = WX * TY > 1;
    if (j < g.ny && x0 < g.nx) {  // uniform per wave
      // Streamed (HBM-bound) sweeps on 64-wide tiles keep the predicated
      // march for full rows too: its wait on each level's store measured
      // faster there.
      if ((!NT || WX > 1) && x0 + 64 <= g.nx)  // uniform per wave
        acc = march_row<true, kShift, CHEB, CHECK, NT>(a, t, lane, i, j);
      else
        acc = march_row<false, kShift, CHEB, CHECK, NT>(a, t, lane, i, j);
    }
  }
  if (a.dec_m >= 0 && blockIdx.x == 0 && threadIdx.x < 64) {
    // The residual test of an earlier checking launch, decided here by one
    // wave after its row instead of by a launch of its own: its partials are
    // complete at this launch's start.  The other blocks sweep regardless;
    // their outputs go to buffers that hold neither the tested iterate nor
    // this launch's input, and the next launch sees the decision.
    double t = 0.0;
#pragma unroll 16
    for (int q = (int)threadIdx.x; q < a.dec_np; q += 64) t += a.dec_partials[q];
    t = wave_sum(t);
    if (threadIdx.x == 0) check_decision(a.ctl, t, a.dec_m);
  }
  if (CHECK) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
  }
}

// --------------------------------------------------------------- 2 sweeps

constexpr int kU2 = 2;  // planes per barrier in the two-sweep kernel

template <typename T, int TY, bool CHEB, bool CHECK>
__global__ __launch_bounds__(64 * TY) void sweep2_kernel(SweepArgs<T> a) {
  if (a.ctl->done) return;
  // First-sweep planes, slot k mod R.  A batch writes kU2 planes and reads
  // kU2 planes starting one below; R = 2 kU2 + 1 keeps the next batch's
  // writes clear of slower threads still reading, with one barrier per batch.
  constexpr int kU = kU2;
  constexpr int R = 2 * kU + 1;
  __shared__ T lvl1[R][TY][64];
  const Grid &g = a.g;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
  double acc = 0.0;
  if (tile < a.ntiles) {
    const TileIdx t = tile_of(tile, a.tiles_x, a.tiles_y, a.kc, g.nz);
    // unwrapped coordinates of this thread's column; the core is
    // lx in [1, 63), ly in [1, TY-1)
    const int xu = t.tx * 62 - 1 + lx, yu = t.ty * (TY - 2) - 1 + ly;
    const bool core = lx >= 1 && lx < 63 && ly >= 1 && ly < TY - 1 && xu < g.nx && yu < g.ny;
    const int i = pmod(xu, g.nx), j = pmod(yu, g.ny);
    const int ip = i + 1 == g.nx ? 0 : i + 1, im = i == 0 ? g.nx - 1 : i - 1;
    const int jp = j + 1 == g.ny ? 0 : j + 1, jm = j == 0 ? g.ny - 1 : j - 1;
    const int64_t col = (int64_t)i + (int64_t)g.nx * j;
    const int64_t oxp = ip - i, oxm = im - i;
    const int64_t oyp = (int64_t)(jp - j) * g.nx, oym = (int64_t)(jm - j) * g.nx;
    const bool cheb1 = CHEB && !a.first, cheb2 = CHEB;
    // first-sweep planes [kb, ke]; second sweep on [k0, k1)
    const int kb = max(0, t.k0 - 1), ke = min(g.nz - 1, t.k1);
    T below = a.cur[col + g.nxy * (kb > 0 ? kb - 1 : 0)];
    T c = a.cur[col + g.nxy * kb];
    // own-column values of the two planes below the current batch
    T l1_m1 = T(0), l1_m2 = T(0), c_m1 = T(0), r_m1 = T(0);
    for (int kbase = kb; kbase <= ke; kbase += kU) {
      const int nb = min(kU, ke - kbase + 1);
      T ab[kU], xp[kU], xm[kU], yp[kU], ym[kU], rr[kU], pp[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (u < nb) {
          const int k = kbase + u;
          const int64_t q = col + g.nxy * k;
          ab[u] = a.cur[q + (k + 1 < g.nz ? g.nxy : 0)];
          xp[u] = a.cur[q + oxp];
          xm[u] = a.cur[q + oxm];
          yp[u] = a.cur[q + oyp];
          ym[u] = a.cur[q + oym];
          rr[u] = a.rhs[q];
          pp[u] = cheb1 ? a.prev[q] : T(0);
        }
      }
      // ---- first sweep on planes kbase .. kbase+nb-1 (whole 64 x TY tile)
      T l1v[kU], cv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        l1v[u] = T(0);
        cv[u] = T(0);
        if (u < nb) {
          const int k = kbase + u;
          const int64_t q = col + g.nxy * k;
          const double hx = (double)xp[u] + (double)xm[u];
          const double hy = (double)yp[u] + (double)ym[u];
          const double hz = (double)ab[u] + (double)below;
          const double res = point_residual(a.k, (double)c, hx, hy, hz, (double)rr[u]);
          const bool core_plane = k >= t.k0 && k < t.k1;
          if (CHECK && core && core_plane) acc += res * res;
          const T l1 = (T)point_update(a.k, (double)c, res, cheb1, (double)pp[u], a.wc0);
          lvl1[k % R][ly][lx] = l1;
          if (CHEB && core && core_plane) a.out_prev[q] = l1;
          l1v[u] = l1;
          cv[u] = c;
          below = c;
          c = ab[u];
        }
      }
      __syncthreads();
      // ---- second sweep on planes kk = kbase-1+u, u = 0 .. nb (the last
      // one only for the top level), core columns only
#pragma unroll
      for (int u = 0; u <= kU; ++u) {
        const int kk = kbase - 1 + u;
        const bool valid = u < nb || (u == nb && kk == g.nz - 1);
        if (!valid || !core || kk < t.k0 || kk >= t.k1) continue;
        const T ctr = u == 0 ? l1_m1 : l1v[u - 1 < 0 ? 0 : u - 1];
        const T lo = kk == 0 ? ctr : (u == 0 ? l1_m2 : (u == 1 ? l1_m1 : l1v[u - 2 < 0 ? 0 : u - 2]));
        const T hi = kk + 1 == g.nz ? ctr : l1v[u < kU ? u : kU - 1];
        const T *pl = &lvl1[kk % R][0][0];
        const double h2x = (double)pl[ly * 64 + lx + 1] + (double)pl[ly * 64 + lx - 1];
        const double h2y = (double)pl[(ly + 1) * 64 + lx] + (double)pl[(ly - 1) * 64 + lx];
        const double h2z = (double)hi + (double)lo;
        const double r2 = u == 0 ? (double)r_m1 : (double)rr[u - 1 < 0 ? 0 : u - 1];
        const double pv2 = u == 0 ? (double)c_m1 : (double)cv[u - 1 < 0 ? 0 : u - 1];
        const double res2 = point_residual(a.k, (double)ctr, h2x, h2y, h2z, r2);
        a.out_last[col + g.nxy * kk] = (T)point_update(a.k, (double)ctr, res2, cheb2, pv2, a.wc1);
      }
      // history for the next batch (compile-time indices only)
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (u == nb - 1) {
          l1_m2 = u >= 1 ? l1v[u >= 1 ? u - 1 : 0] : l1_m1;
          l1_m1 = l1v[u];
          c_m1 = cv[u];
          r_m1 = rr[u];
        }
      }
    }
  }
  if (CHECK) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
  }
}

constexpr int kTY2 = 8;  // two-sweep tile: 512 threads, core 62 x 6

struct Shape {
  int kc, tiles_x, tiles_y, tiles_z, ntiles, blocks;
  int wx, ty;   // one-sweep kernel: waves along x, tile rows
  bool stream;  // one-sweep kernel: streamed arrays
};

// The four arrays of a sweep exceed what the Infinity Cache keeps.
bool streamed(const Grid &g, bool is_double) {
  return 4.0 * (double)g.n * (is_double ? 8.0 : 4.0) > 192.0e6;
}

Shape shape_of(const Grid &g, int S, bool is_double) {
  Shape sh;
  sh.stream = S == 1 && streamed(g, is_double);
  sh.wx = 1;
  sh.ty = 0;
  if (S == 1) {
    int ty;
    if (g.nx >= kWideNx && g.ny >= kWideTYBig) {
      sh.wx = kWX;
      ty = sh.stream ? kWideTYBig : kWideTY;
    } else {
      // rows beyond ny would idle: a short y axis (a two-dimensional run
      // has ny = 1) takes the next smaller tile
      ty = sh.stream ? kTY1Big : kTY1;
      if (g.ny < ty) ty = g.ny < kTY1 ? 1 : kTY1;
    }
    sh.ty = ty;
    sh.tiles_x = (g.nx + 64 * sh.wx - 1) / (64 * sh.wx);
    sh.tiles_y = (g.ny + ty - 1) / ty;
  } else {
    sh.tiles_x = (g.nx + 61) / 62;
    sh.tiles_y = (g.ny + kTY2 - 3) / (kTY2 - 2);
  }
  const int64_t cols = (int64_t)sh.tiles_x * sh.tiles_y;
  // z chunks: long enough to amortise the halo planes, short enough for
  // several blocks per CU.  Wide tiles aim at a wave count: the 8192 waves
  // that fill the chip once when cache-resident, eight times that when
  // streamed (shorter chunks measured faster there).
  sh.kc = g.nz;
  const int target = sh.wx > 1 ? (sh.stream ? 65536 : 8192) / (sh.wx * sh.ty) : 2048;
  while (sh.kc > 8 && cols * ((g.nz + sh.kc - 1) / sh.kc) < target) sh.kc = (sh.kc + 1) / 2;
  sh.tiles_z = (g.nz + sh.kc - 1) / sh.kc;
  int64_t nt = cols * sh.tiles_z;
  while (nt > kPartials) {
    sh.kc *= 2;
    sh.tiles_z = (g.nz + sh.kc - 1) / sh.kc;
    nt = cols * sh.tiles_z;
  }
  sh.ntiles = (int)nt;
  sh.blocks = (sh.ntiles + 7) / 8 * 8;
  return sh;
}

}  // namespace

int tsweep_blocks(const Grid &g, int S, bool is_double) {
  return shape_of(g, S, is_double).blocks;
}

template <typename T>
void launch_tsweep(const Grid &g, int S, bool chebyshev, bool check, bool first,
                   double omega_jacobi, const double *omega_cheb, const T *cur, const T *prev,
                   T *out_last, T *out_prev, const T *rhs, SolveCtl *ctl, double *partials,
                   const double *dec_partials, int dec_np, int dec_m, hipStream_t s) {
  const Shape sh = shape_of(g, S, sizeof(T) == 8);
  SweepArgs<T> a;
  a.g = g;
  a.k.ix2 = 1.0 / (g.dx * g.dx);
  a.k.iy2 = 1.0 / (g.dy * g.dy);
  a.k.iz2 = 1.0 / (g.dz * g.dz);
  a.k.diag = 2.0 * (a.k.ix2 + a.k.iy2 + a.k.iz2);
  a.k.inv_diag = 1.0 / a.k.diag;
  a.k.omega_j = omega_jacobi;
  a.kc = sh.kc;
  a.tiles_x = sh.tiles_x;
  a.tiles_y = sh.tiles_y;
  a.tiles_z = sh.tiles_z;
  a.ntiles = sh.ntiles;
  a.wc0 = omega_cheb[0];
  a.wc1 = S > 1 ? omega_cheb[1] : 1.0;
  a.first = first ? 1 : 0;
  a.cur = cur;
  a.prev = prev;
  a.rhs = rhs;
  a.out_last = out_last;
  a.out_prev = out_prev;
  a.ctl = ctl;
  a.partials = partials;
  a.dec_partials = dec_partials;
  a.dec_np = dec_np;
  a.dec_m = S == 1 ? dec_m : -1;
  const dim3 grid(sh.blocks);
#define LES_PICK(WX, TY, NT)                                                          \
  do {                                                                                \
    const dim3 block(64 * WX * TY);                                                   \
    if (chebyshev && !first) {                                                        \
      if (check) sweep1_kernel<T, WX, TY, true, true, NT><<<grid, block, 0, s>>>(a);  \
      else sweep1_kernel<T, WX, TY, true, false, NT><<<grid, block, 0, s>>>(a);       \
    } else {                                                                          \
      if (check) sweep1_kernel<T, WX, TY, false, true, NT><<<grid, block, 0, s>>>(a); \
      else sweep1_kernel<T, WX, TY, false, false, NT><<<grid, block, 0, s>>>(a);      \
    }                                                                                 \
  } while (0)
  if (S == 1) {
    if (sh.wx == kWX && sh.stream)
      LES_PICK(kWX, kWideTYBig, true);
    else if (sh.wx == kWX)
      LES_PICK(kWX, kWideTY, false);
    else if (sh.ty == kTY1Big)
      LES_PICK(1, kTY1Big, true);
    else if (sh.ty == kTY1 && !sh.stream)
      LES_PICK(1, kTY1, false);
    else if (sh.ty == kTY1)
      LES_PICK(1, kTY1, true);
    else if (!sh.stream)
      LES_PICK(1, 1, false);
    else
      LES_PICK(1, 1, true);
  } else {
    const dim3 block(64 * kTY2);
    if (chebyshev) {
      if (check) sweep2_kernel<T, kTY2, true, true><<<grid, block, 0, s>>>(a);
      else sweep2_kernel<T, kTY2, true, false><<<grid, block, 0, s>>>(a);
    } else {
      if (check) sweep2_kernel<T, kTY2, false, true><<<grid, block, 0, s>>>(a);
      else sweep2_kernel<T, kTY2, false, false><<<grid, block, 0, s>>>(a);
    }
  }
#undef LES_PICK
}

template void launch_tsweep<float>(const Grid &, int, bool, bool, bool, double, const double *,
                                   const float *, const float *, float *, float *, const float *,
                                   SolveCtl *, double *, const double *, int, int, hipStream_t);
template void launch_tsweep<double>(const Grid &, int, bool, bool, bool, double, const double *,
                                    const double *, const double *, double *, double *,
                                    const double *, SolveCtl *, double *, const double *, int, int,
                                    hipStream_t);

}  // namespace lesmi
