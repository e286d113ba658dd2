// Plane-staged stencil access for the z-marching kernels.
//
// A block owns a kTileX x kTileY tile of columns and marches a chunk of z
// levels.  At each level the x-y neighbourhoods of the stencil fields come
// from LDS planes (the tile plus a ring of H cells, sources wrapped
// periodically), the z neighbourhoods of the block's own columns from
// values carried up the march in registers.  So each cell of a field is
// read from memory about once per level (plus the ring, which neighbouring
// tiles read as well and which the XCD's L2 serves), however many stencil
// points use it.  Threads run along x first (a wave is 64 consecutive
// columns of a row); tiles past the grid's edge compute on wrapped columns
// and store nothing there.
#pragma once

#include <type_traits>
#include <utility>

#include "les_device.h"

namespace lesmi {

constexpr int kTileX = 64, kTileY = 8;
constexpr int kTileThreads = kTileX * kTileY;
constexpr int kTileDepth = 4;  // levels the loads of a march run ahead

// Launch of a tiled z march: tiles of kTileX x kTileY columns, each column
// split into z chunks of kc levels, halved from the whole column (to 8
// levels at least) until there are ~2 blocks per CU (longer chunks re-read
// fewer halo levels and refill fewer register FIFOs; the kernels hide
// memory latency by loading several levels ahead); the grid is a multiple
// of 8 blocks (see tile_of).
struct TileMap {
  int tiles_x, tiles_y, kc, nkc, tiles;
  unsigned blocks;
};
inline TileMap tile_map(const Grid &g) {
  TileMap m;
  m.tiles_x = (g.nx + kTileX - 1) / kTileX;
  m.tiles_y = (g.ny + kTileY - 1) / kTileY;
  const int64_t cols = (int64_t)m.tiles_x * m.tiles_y;
  m.kc = g.nz;
  while (m.kc > 8 && cols * ((g.nz + m.kc - 1) / m.kc) < 512) m.kc = (m.kc + 1) / 2;
  m.nkc = (g.nz + m.kc - 1) / m.kc;
  m.tiles = (int)(cols * m.nkc);
  m.blocks = (unsigned)((m.tiles + 7) / 8 * 8);
  return m;
}

// The block's tile: XCD x (blocks b with b % 8 = x) takes the x-th
// contiguous range of tiles in the order x tile, y tile, z chunk, so that
// neighbouring tiles (which read each other's edge rows as their ring) run
// on one XCD.
struct Tile {
  int x0, y0, k0, k1;
  bool valid;
};
__device__ __forceinline__ Tile tile_of(const Grid &g, const TileMap &m) {
  const int per = (int)(gridDim.x >> 3);
  int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  Tile T;
  T.valid = t < m.tiles;
  if (!T.valid) t = 0;
  const int tx = t % m.tiles_x;
  t /= m.tiles_x;
  const int ty = t % m.tiles_y;
  const int kz = t / m.tiles_y;
  T.x0 = tx * kTileX;
  T.y0 = ty * kTileY;
  T.k0 = kz * m.kc;
  T.k1 = min(g.nz, T.k0 + m.kc);
  return T;
}

__device__ __forceinline__ int wrap_mod(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// The calling thread's column (x fastest); its in-plane offset (the
// column wrapped into the grid) and whether it lies inside the grid.
struct TileCol {
  int lx, ly;
  int64_t off;
  bool active;
};
__device__ __forceinline__ TileCol tile_col(const Grid &g, const Tile &T) {
  TileCol c;
  c.lx = (int)(threadIdx.x % kTileX);
  c.ly = (int)(threadIdx.x / kTileX);
  const int i = T.x0 + c.lx, j = T.y0 + c.ly;
  c.active = i < g.nx && j < g.ny;
  c.off = (int64_t)wrap_mod(i, g.nx) + (int64_t)g.nx * wrap_mod(j, g.ny);
  return c;
}

// One field's LDS plane: the tile plus a ring of HX cells left and right
// of its rows and HY cells above and below its columns (the stencils are
// axis-aligned, so the corners are not held).  Cell (py, px) holds column
// (x0 - HX + px, y0 - HY + py), wrapped.
template <typename T, int HX, int HY>
struct TilePlane {
  static constexpr int PX = kTileX + 2 * HX, PY = kTileY + 2 * HY;
  T v[PY][PX];
};

// The ring cells a thread loads: ring cell h of a plane (the HY rows above
// and below the tile's columns, then HX cells left and right of its rows),
// for h = thread + kTileThreads u.  src: in-plane offset of the column
// (wrapped), -1 past the ring; dst: flat index py PX + px.
template <int HX, int HY>
struct RingCells {
  static constexpr int PX = kTileX + 2 * HX;
  static constexpr int N = 2 * HY * kTileX + 2 * HX * kTileY;
  static constexpr int PER = (N + kTileThreads - 1) / kTileThreads;
  int64_t src[PER];
  int dst[PER];
};
template <int HX, int HY>
__device__ __forceinline__ RingCells<HX, HY> ring_cells(const Grid &g, const Tile &T) {
  using R = RingCells<HX, HY>;
  R r;
#pragma unroll
  for (int u = 0; u < R::PER; ++u) {
    const int h = (int)threadIdx.x + kTileThreads * u;
    int py = 0, px = 0;
    if (h < HY * kTileX) {  // rows above the tile
      py = h / kTileX;
      px = HX + h % kTileX;
    } else if (h < 2 * HY * kTileX) {  // rows below
      const int hh = h - HY * kTileX;
      py = HY + kTileY + hh / kTileX;
      px = HX + hh % kTileX;
    } else if constexpr (HX > 0) {  // left and right of the tile's rows
      const int hh = h - 2 * HY * kTileX;
      const int c = hh % (2 * HX);
      py = HY + hh / (2 * HX);
      px = c < HX ? c : kTileX + c;
    }
    const bool in = h < R::N;
    r.dst[u] = in ? py * R::PX + px : -1;
    r.src[u] = in ? (int64_t)wrap_mod(T.x0 - HX + px, g.nx) +
                        (int64_t)g.nx * wrap_mod(T.y0 - HY + py, g.ny)
                  : -1;
  }
  return r;
}

// Value of column `off` of field f at level kk (z ghost levels: the
// mirrored level times the field's parity).
template <typename T>
__device__ __forceinline__ T col_value(const Grid &g, const T *__restrict__ f, int64_t off, int kk,
                                       T par) {
  const int km = zmirror(kk, g.nz);
  const T v = f[(int64_t)km * g.nxy + off];
  return km == kk ? v : par * v;
}

// Runs f(std::integral_constant<int, P>{}, k + P) for P = 0, 1, ... while
// k + P < k1: one trip of a z march unrolled by the depth of its register
// FIFOs (so that every FIFO slot is a fixed register).  False when the
// march has ended.
template <class F, int... P>
__device__ __forceinline__ bool march_trip(F &f, int k, int k1, std::integer_sequence<int, P...>) {
  return ((k + P < k1 ? (f(std::integral_constant<int, P>{}, k + P), true) : false) && ...);
}

}  // namespace lesmi
