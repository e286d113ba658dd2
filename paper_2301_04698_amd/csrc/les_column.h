// Column-marching stencil access for the advection, diffusion, divergence
// and projection kernels.
//
// A wave owns one 64-cell row segment along x of one y row and marches a
// chunk of z levels.  The periodic x/y neighbour offsets of its columns are
// computed once; the level, its wall mirrors and the plane addresses are
// uniform over the wave, so a stencil load is a 32-bit per-lane byte offset
// from a scalar plane address (no per-load index arithmetic), and the wall
// ghosts of the z stencil are resolved by uniform branches on the few levels
// next to the walls.  Neighbouring rows of a block share their y halos in
// the CU's caches, and each XCD gets one contiguous range of row segments.
#pragma once

#include "les_device.h"

namespace lesmi {

constexpr int kColWaves = 4;  // row segments (waves) per block

// Work decomposition of a column-marching launch: units are (y row,
// x segment, z chunk) with the row fastest; four units per block.
struct ColMap {
  int ntx;       // 64-cell x segments per row
  int kc;        // levels per z chunk
  int nkc;       // z chunks
  int units;     // ny * ntx * nkc: at most n / 8, below 2^31 for any grid whose
                 // workspace (25 fields) fits in one GPU's memory
  int blocks;    // multiple of 8 (one contiguous range of blocks per XCD)
};

// Chunks of 16 levels, shortened (to four at least) until the launch has
// about 32768 waves (128 per CU) where the grid allows.  The chunk length
// changes little: 4, 8, 16 and 32 levels at 256x256x128 are within 6 %.
inline ColMap col_map(const Grid &g) {
  ColMap m;
  m.ntx = (g.nx + 63) / 64;
  const int64_t cols = (int64_t)g.ny * m.ntx;
  m.kc = 16;
  while (m.kc > 4 && cols * ((g.nz + m.kc - 1) / m.kc) < 32768) m.kc >>= 1;
  m.nkc = (g.nz + m.kc - 1) / m.kc;
  m.units = (int)(cols * m.nkc);
  const int64_t nb = (m.units + kColWaves - 1) / kColWaves;
  m.blocks = (int)((nb + 7) / 8 * 8);
  return m;
}

// The unit of the calling wave: row j, lane column i (clamped to the grid
// for addressing; `active` marks lanes inside it) and levels [k0, k1).
struct ColWave {
  int i, j, k0, k1;
  bool active, valid;
};

__device__ __forceinline__ ColWave col_wave(const Grid &g, const ColMap &m) {
  const int per = gridDim.x >> 3;
  const int lb = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int u = lb * kColWaves + wave;
  ColWave c;
  c.valid = u < m.units;
  const int r = u / g.ny;
  c.j = u - r * g.ny;
  const int tx = r % m.ntx;
  const int kc = r / m.ntx;
  c.k0 = kc * m.kc;
  c.k1 = min(c.k0 + m.kc, g.nz);
  const int i = tx * 64 + (int)(threadIdx.x & 63);
  c.active = i < g.nx;
  c.i = c.active ? i : g.nx - 1;
  return c;
}

// Byte offsets within a plane of the columns (i + di, j + dj), |di|, |dj|
// <= 2, periodic (a y axis of one cell has a zero row stride).  A plane is
// at most 2 GiB (checked when the library is set up).
template <typename T>
struct ColPts {
  uint32_t o[5][5];
};

template <typename T>
__device__ __forceinline__ ColPts<T> col_pts(const Grid &g, int i, int j) {
  ColPts<T> p;
  const uint32_t sy = (uint32_t)g.sy;
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b)
      p.o[a][b] = ((uint32_t)pwrap(i + a - 2, g.nx) + sy * (uint32_t)pwrap(j + b - 2, g.ny)) *
                  (uint32_t)sizeof(T);
  return p;
}

// Buffer resource of one z plane of a field: base address of the plane,
// its size in bytes as the range, raw (unformatted) access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *f, int64_t pb, int z) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char *>(reinterpret_cast<const char *>(f) + z * pb), (short)0, (int)pb,
      0x00020000);
}

template <typename T>
__device__ __forceinline__ T rsrc_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void rsrc_store(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) uint32_t, v), r, (int)off, 0, 0);
}

// Stencil access at level k of a wave's columns: plane address (scalar)
// plus the lane's column offset (loop-invariant vector register), no
// per-load address arithmetic.  EDGE: the level is within two cells of a
// wall, so z neighbours may be ghosts (the mirrored level, times the
// field's parity).
template <typename T, bool EDGE>
struct Lvl {
  const ColPts<T> &p;
  int k;
  int64_t pb;  // bytes per plane
  int zk[5];   // level of k + dk after the wall mirror, dk in [-2, 2]

  __device__ __forceinline__ Lvl(const Grid &g, const ColPts<T> &pts, int k_)
      : p(pts), k(k_), pb(g.nxy * (int64_t)sizeof(T)) {
#pragma unroll
    for (int dk = -2; dk <= 2; ++dk) zk[dk + 2] = EDGE ? zmirror(k + dk, g.nz) : k + dk;
  }

  // Field f at (i + di, j + dj, k + dk) with ghost parity par (+1 even,
  // -1 odd); offsets are compile-time after inlining.
  __device__ __forceinline__ T operator()(const T *__restrict__ f, int di, int dj, int dk,
                                          T par) const {
    const T v = rsrc_load<T>(plane_rsrc(f, pb, zk[dk + 2]), p.o[di + 2][dj + 2]);
    if (EDGE && par < T(0) && zk[dk + 2] != k + dk) return -v;
    return v;
  }

  // Profile value at k + dk (even extension across the walls).
  __device__ __forceinline__ T prof(const T *__restrict__ a, int dk) const { return a[zk[dk + 2]]; }

  // Store v to the lane's own cell of field f.  Lanes outside the grid
  // store at an offset beyond the plane's range (at least 2 GiB; a plane
  // is at most 2 GiB), which the buffer range check discards: no
  // divergent branch around the store.
  __device__ __forceinline__ void store(T *f, T v, bool active) const {
    rsrc_store<T>(plane_rsrc(f, pb, k), active ? p.o[2][2] : 0x80000000u, v);
  }
};

}  // namespace lesmi
