// Device helpers: boundary-aware loads, wavefront/block FP64 reductions.
#pragma once

#include "les_internal.h"

namespace lesmi {

// Periodic neighbour index for offsets |o| <= 2; one wrap suffices for
// n >= 2.  A y axis of one cell (a two-dimensional run) leaves j in
// [-1, 1], which gload multiplies by a zero row stride.
__device__ __forceinline__ int pwrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Mirror across the walls z = 0 and z = H: level -1 -> 0, -2 -> 1, nz -> nz-1, nz+1 -> nz-2.
__device__ __forceinline__ int zmirror(int k, int nz) {
  return k < 0 ? -1 - k : (k >= nz ? 2 * nz - 1 - k : k);
}

// Value of a cell-centred field at (i, j, k) with ghost cells: periodic x/y,
// wall mirror in z times the field's parity (+1 even: scalars, pressure,
// viscosity, buoyancy; -1 odd: velocity components).
template <typename T>
__device__ __forceinline__ T gload(const T *__restrict__ f, const Grid &g, int i, int j, int k,
                                   T parity) {
  i = pwrap(i, g.nx);
  j = pwrap(j, g.ny);
  int km = zmirror(k, g.nz);
  T v = f[(int64_t)i + g.sy * j + g.nxy * km];
  return km == k ? v : parity * v;
}

// Profile value with even extension across the walls.
template <typename T>
__device__ __forceinline__ T pload(const T *__restrict__ a, int k, int nz) {
  return a[zmirror(k, nz)];
}

// Rows of a row-wise pass over a grid of a multiple of 8 blocks: XCD x
// (the blocks b with b % 8 = x) takes the x-th contiguous eighth of the
// rows and each of its blocks a consecutive run of them, so that the rows
// beside a row (y +- 1 in the same run, z +- 1 one level of rows away) are
// read on one XCD close in time and come from its L2.
struct RowRange {
  int64_t r0, r1;
};
__device__ __forceinline__ RowRange xcd_rows(int64_t rows) {
  const int64_t per = gridDim.x >> 3, rpx = (rows + 7) / 8, rpb = (rpx + per - 1) / per;
  const int64_t x = blockIdx.x & 7, lb = blockIdx.x >> 3;
  const int64_t lo = x * rpx + lb * rpb;
  RowRange r;
  r.r0 = lo < rows ? lo : rows;
  r.r1 = min(min(lo + rpb, (x + 1) * rpx), rows);
  if (r.r1 < r.r0) r.r1 = r.r0;
  return r;
}

// Level k and y row j of the x row r = k ny + j, and stepping r by a
// fixed stride without divisions (the stride's quotient and remainder by
// ny are formed once).
struct RowPos {
  int k, j;
};
struct RowStep {
  int ny, sk, sj;
  __device__ __forceinline__ RowStep(int ny_, int64_t stride)
      : ny(ny_), sk((int)(stride / ny_)), sj((int)(stride - (stride / ny_) * ny_)) {}
  __device__ __forceinline__ RowPos at(int64_t r) const {
    RowPos p;
    p.k = (int)(r / ny);
    p.j = (int)(r - (int64_t)p.k * ny);
    return p;
  }
  __device__ __forceinline__ RowPos next(RowPos p) const {
    p.k += sk;
    p.j += sj;
    if (p.j >= ny) {
      p.j -= ny;
      ++p.k;
    }
    return p;
  }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide FP64 sum (blockDim.x a multiple of 64, at most 1024 threads).
// Result valid in thread 0.  Fixed order: deterministic for a fixed launch.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[16];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) s += red[q];
  }
  __syncthreads();
  return s;
}

// Stopping decision of the residual check at sweep m with squared residual
// norm s (one thread): converged when s <= tol^2 ||rhs||^2, non-finite, or
// the sweep cap; a fixed-count solve stops only at its count.
__device__ __forceinline__ void check_decision(SolveCtl *ctl, double s, int m) {
  if (ctl->done) return;
  ctl->res_norm2 = s;
  if (!isfinite(s)) {
    ctl->done = 2;
    ctl->stop_m = m;
  } else if (ctl->fixed) {
    if (m >= ctl->max_sweeps) {
      ctl->done = s <= ctl->tol2 ? 1 : 3;
      ctl->stop_m = m;
    }
  } else if (s <= ctl->tol2) {
    ctl->done = 1;
    ctl->stop_m = m;
  } else if (m >= ctl->max_sweeps) {
    ctl->done = 3;
    ctl->stop_m = m;
  }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Block-wide maximum (same launch constraints as block_sum).
__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[16];
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = v;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int q = 0; q < nw; ++q) s = fmax(s, red[q]);
  }
  __syncthreads();
  return s;
}

}  // namespace lesmi
