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
// Two sweeps: one wave per four rows and 62-cell segment also forms the
// first sweep of the two rows beside them in registers, so the second sweep
// needs no LDS and no barrier; 20 bytes per cell from memory for both
// sweeps (phi, prev, rhs in; the two new iterates out).
//
// Walls: the z neighbour of the bottom/top level is that level itself (even
// mirror); x and y are periodic.
#include "les_column.h"

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
  // host-visible word written after that decision (device view of pinned
  // host memory; nullable): decision number snap_seq in the high half, the
  // control block's `done` in the low half, one 64-bit store
  int64_t *snap;
  int snap_seq;
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
  if (a.ctl->done) {  // stopped: a deciding launch still leaves its word
    if (a.snap && blockIdx.x == 0 && threadIdx.x == 0)
      *(volatile int64_t *)a.snap = ((int64_t)a.snap_seq << 32) | (uint32_t)a.ctl->done;
    return;
  }
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
    if (threadIdx.x == 0) {
      check_decision(a.ctl, t, a.dec_m);
      if (a.snap)
        *(volatile int64_t *)a.snap = ((int64_t)a.snap_seq << 32) | (uint32_t)a.ctl->done;
    }
  }
  if (CHECK) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
  }
}

// --------------------------------------------------------------- 2 sweeps

// Two fused sweeps without LDS or barriers.  A wave owns R rows j0 ..
// j0+R-1 and a 62-cell x segment (lanes 1..62; lanes 0 and 63 are its halo
// columns, wrapped periodically like every other lane) of the z chunk
// [k0, k1).  Marching up z it forms the first sweep on rows j0-1 .. j0+R at
// level k (their y neighbours are rows j0-2 .. j0+R+1 of the iterate, x
// neighbours the adjacent lanes, z neighbours registers), then the second
// sweep on its R rows at level k-1 from first-sweep values that are all in
// its own registers or adjacent lanes.  The first sweep of the two boundary
// rows is also formed by the neighbouring waves; in exchange every array is
// read from memory once per two sweeps (neighbour rows through the caches).
// All accesses are buffer loads and stores on one z plane: lanes outside
// the segment's core, and rows beyond the grid, store at an offset past the
// plane's range, which the hardware drops.
constexpr int kR2 = 4;  // rows per wave of the two-sweep kernel

template <typename T, int R, bool CHEB, bool CHECK>
__global__ __launch_bounds__(256) void sweep2_kernel(SweepArgs<T> a) {
  if (a.ctl->done) return;
  constexpr int NR = R + 2;  // first-sweep rows j0-1 .. j0+R
  const Grid &g = a.g;
  const int lb = xcd_tile(blockIdx.x, gridDim.x);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  const int u = lb * 4 + wave;
  double acc = 0.0;
  if (u < a.ntiles) {  // uniform per wave
    const int ty = u % a.tiles_y, rest = u / a.tiles_y;
    const int tx = rest % a.tiles_x, tz = rest / a.tiles_x;
    const int j0 = ty * R;
    const int k0 = tz * a.kc, k1 = min(g.nz, k0 + a.kc);
    const int xu = tx * 62 - 1 + lane;
    const bool core = lane >= 1 && lane <= 62 && xu < g.nx;
    const int i = pmod(xu, g.nx), il = pmod(xu - 1, g.nx), ir = pmod(xu + 1, g.nx);
    constexpr uint32_t kOut = 0x80000000u;  // beyond any plane (at most 2 GiB)
    const uint32_t es = (uint32_t)sizeof(T);
    uint32_t o[R + 4];  // rows j0-2 .. j0+R+1 of this lane's column
#pragma unroll
    for (int d = 0; d < R + 4; ++d)
      o[d] = ((uint32_t)i + (uint32_t)g.nx * (uint32_t)pmod(j0 + d - 2, g.ny)) * es;
    uint32_t oxl[NR], oxr[NR];  // x neighbours of the end lanes
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      const uint32_t row = (uint32_t)g.nx * (uint32_t)pmod(j0 + d - 1, g.ny);
      oxl[d] = lane == 0 ? ((uint32_t)il + row) * es : kOut;
      oxr[d] = lane == 63 ? ((uint32_t)ir + row) * es : kOut;
    }
    uint32_t ost[R];  // store offsets of the output rows
    bool rcore[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      rcore[r] = core && j0 + r < g.ny;
      ost[r] = rcore[r] ? o[r + 2] : kOut;
    }
    const int64_t pb = g.nxy * (int64_t)sizeof(T);
    const bool cheb1 = CHEB && !a.first;
    const int kb = max(0, k0 - 1), ke = min(g.nz - 1, k1);
    // iterate of the first-sweep rows at levels k-1 (bl) and k (cc)
    T bl[NR], cc[NR];
    {
      const __amdgpu_buffer_rsrc_t rb = plane_rsrc(a.cur, pb, kb > 0 ? kb - 1 : 0);
      const __amdgpu_buffer_rsrc_t rc = plane_rsrc(a.cur, pb, kb);
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        bl[d] = rsrc_load<T>(rb, o[d + 1]);
        cc[d] = rsrc_load<T>(rc, o[d + 1]);
      }
    }
    // first-sweep values at level k-1 (all rows) and k-2 (output rows);
    // rhs and iterate of the output rows at level k-1
    T s1p[NR], s1pp[R], rm1[R], cm1[R];
#pragma unroll
    for (int d = 0; d < NR; ++d) s1p[d] = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) s1pp[r] = rm1[r] = cm1[r] = T(0);
    for (int k = kb; k <= ke; ++k) {
      const __amdgpu_buffer_rsrc_t rk = plane_rsrc(a.cur, pb, k);
      const __amdgpu_buffer_rsrc_t ra = plane_rsrc(a.cur, pb, k + 1 < g.nz ? k + 1 : k);
      const __amdgpu_buffer_rsrc_t rr = plane_rsrc(a.rhs, pb, k);
      T ab[NR], rh[NR], pv[NR], xl[NR], xr[NR];
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        ab[d] = rsrc_load<T>(ra, o[d + 1]);
        rh[d] = rsrc_load<T>(rr, o[d + 1]);
        xl[d] = rsrc_load<T>(rk, oxl[d]);
        xr[d] = rsrc_load<T>(rk, oxr[d]);
        pv[d] = T(0);
      }
      const T ylo = rsrc_load<T>(rk, o[0]), yhi = rsrc_load<T>(rk, o[R + 3]);
      if (cheb1) {
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(a.prev, pb, k);
#pragma unroll
        for (int d = 0; d < NR; ++d) pv[d] = rsrc_load<T>(rp, o[d + 1]);
      }
      const bool core_k = k >= k0 && k < k1;
      // ---- first sweep, rows j0-1 .. j0+R at level k
      T s1[NR];
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        const T sp = lane_shift<1>(cc[d]), sm = lane_shift<-1>(cc[d]);
        const T xp = lane == 63 ? xr[d] : sp;
        const T xm = lane == 0 ? xl[d] : sm;
        const T yp = d == NR - 1 ? yhi : cc[d < NR - 1 ? d + 1 : NR - 1];
        const T ym = d == 0 ? ylo : cc[d > 0 ? d - 1 : 0];
        const double hx = (double)xp + (double)xm;
        const double hy = (double)yp + (double)ym;
        const double hz = (double)ab[d] + (double)bl[d];
        const double res = point_residual(a.k, (double)cc[d], hx, hy, hz, (double)rh[d]);
        if (CHECK && d >= 1 && d <= R && core_k && rcore[d >= 1 && d <= R ? d - 1 : 0])
          acc += res * res;
        s1[d] = (T)point_update(a.k, (double)cc[d], res, cheb1, (double)pv[d], a.wc0);
      }
      if (CHEB && core_k) {
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.out_prev, pb, k);
#pragma unroll
        for (int r = 0; r < R; ++r) rsrc_store<T>(ro, ost[r], s1[r + 1]);
      }
      // ---- second sweep, output rows at level k-1
      if (k - 1 >= k0 && k - 1 < k1) {
        const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.out_last, pb, k - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T ctr = s1p[r + 1];
          const T lo = k - 1 == 0 ? ctr : s1pp[r];
          const double h2x = (double)lane_shift<1>(ctr) + (double)lane_shift<-1>(ctr);
          const double h2y = (double)s1p[r + 2] + (double)s1p[r];
          const double h2z = (double)s1[r + 1] + (double)lo;
          const double r2 = point_residual(a.k, (double)ctr, h2x, h2y, h2z, (double)rm1[r]);
          rsrc_store<T>(ro, ost[r], (T)point_update(a.k, (double)ctr, r2, CHEB, (double)cm1[r], a.wc1));
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        s1pp[r] = s1p[r + 1];
        rm1[r] = rh[r + 1];
        cm1[r] = cc[r + 1];
      }
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        s1p[d] = s1[d];
        bl[d] = cc[d];
        cc[d] = ab[d];
      }
    }
    if (k1 == g.nz) {  // the top level: its upper neighbour is itself
      const int kk = g.nz - 1;
      const __amdgpu_buffer_rsrc_t ro = plane_rsrc(a.out_last, pb, kk);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T ctr = s1p[r + 1];
        const T lo = kk == 0 ? ctr : s1pp[r];
        const double h2x = (double)lane_shift<1>(ctr) + (double)lane_shift<-1>(ctr);
        const double h2y = (double)s1p[r + 2] + (double)s1p[r];
        const double h2z = (double)ctr + (double)lo;
        const double r2 = point_residual(a.k, (double)ctr, h2x, h2y, h2z, (double)rm1[r]);
        rsrc_store<T>(ro, ost[r], (T)point_update(a.k, (double)ctr, r2, CHEB, (double)cm1[r], a.wc1));
      }
    }
  }
  if (CHECK) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = s;
  }
}

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
    // one wave per kR2 rows and 62-cell x segment, four waves per block; z
    // chunks halved (to 8 levels at least) until about 8192 waves
    sh.tiles_x = (g.nx + 61) / 62;
    sh.tiles_y = (g.ny + kR2 - 1) / kR2;
    const int64_t rows = (int64_t)sh.tiles_x * sh.tiles_y;
    sh.kc = g.nz;
    while (sh.kc > 8 && rows * ((g.nz + sh.kc - 1) / sh.kc) < 8192) sh.kc = (sh.kc + 1) / 2;
    for (;;) {
      sh.tiles_z = (g.nz + sh.kc - 1) / sh.kc;
      if ((rows * sh.tiles_z + 3) / 4 <= kPartials) break;
      sh.kc *= 2;
    }
    sh.ntiles = (int)(rows * sh.tiles_z);
    sh.blocks = ((sh.ntiles + 3) / 4 + 7) / 8 * 8;
    return sh;
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
                   const double *dec_partials, int dec_np, int dec_m, int64_t *snap,
                   int snap_seq, hipStream_t s) {
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
  a.snap = a.dec_m >= 0 ? snap : nullptr;
  a.snap_seq = snap_seq;
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
    const dim3 block(256);
    if (chebyshev) {
      if (check) sweep2_kernel<T, kR2, true, true><<<grid, block, 0, s>>>(a);
      else sweep2_kernel<T, kR2, true, false><<<grid, block, 0, s>>>(a);
    } else {
      if (check) sweep2_kernel<T, kR2, false, true><<<grid, block, 0, s>>>(a);
      else sweep2_kernel<T, kR2, false, false><<<grid, block, 0, s>>>(a);
    }
  }
#undef LES_PICK
}

template void launch_tsweep<float>(const Grid &, int, bool, bool, bool, double, const double *,
                                   const float *, const float *, float *, float *, const float *,
                                   SolveCtl *, double *, const double *, int, int, int64_t *, int,
                                   hipStream_t);
template void launch_tsweep<double>(const Grid &, int, bool, bool, bool, double, const double *,
                                    const double *, const double *, double *, double *,
                                    const double *, SolveCtl *, double *, const double *, int, int,
                                    int64_t *, int, hipStream_t);

}  // namespace lesmi
