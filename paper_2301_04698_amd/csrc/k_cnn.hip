// Guess network kernels: inference of the learned Poisson initial guess and
// the forward/backward/update kernels that train it on solver-generated
// pairs.
//
// Layouts: single-channel fields are (batch, nz, ny, nx) with x fastest;
// network inputs of C channels are (batch, C, nz, ny, nx) in FP32 and
// channels-last bfloat16 (cell * C + c) once rounded; 16-channel
// activations are channels-last bfloat16 (cell * 16 + c), so one cell's
// channels are one 32-byte line.  The two 16 -> 16 layers run on the matrix
// cores as an implicit GEMM per tap: D(out ch x 16 cells) += W_tap(out x
// in) * X_tap(in x 16 cells), FP32 accumulation, one wave per 16
// consecutive output cells; the C -> 16 layer as one GEMM over (tap,
// channel) pairs.  The 16 -> 1 layer and the backward pass are FP32 vector
// code (FP64 sums in the weight gradient).
#include <cmath>

#include "cnn_internal.h"
#include "les_device.h"

namespace lesmi {

CnnGeom cnn_geom(int batch, int nz, int ny, int nx, int periodic, int layer, int inputs) {
  CnnGeom G;
  G.inputs = inputs;
  const int ti = periodic ? 0 : 2 * layer, to = periodic ? 0 : 2 * (layer + 1);
  G.batch = batch;
  G.nz = nz;
  G.nyi = ny - ti;
  G.nxi = nx - ti;
  G.nyo = ny - to;
  G.nxo = nx - to;
  G.periodic = periodic;
  G.n_in = (int64_t)batch * nz * G.nyi * G.nxi;
  G.n_out = (int64_t)batch * nz * G.nyo * G.nxo;
  return G;
}

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// FP32 -> bfloat16, round to nearest, ties to even (finite values): add
// 0x7FFF plus the lowest kept bit, then truncate to the high half.
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float leaky(float v, float alpha) { return v >= 0.f ? v : alpha * v; }

struct Cell {
  int b, k, j, i;
};
__device__ __forceinline__ Cell decode(int64_t q, int nz, int ny, int nx) {
  Cell c;
  c.i = (int)(q % nx);
  q /= nx;
  c.j = (int)(q % ny);
  q /= ny;
  c.k = (int)(q % nz);
  c.b = (int)(q / nz);
  return c;
}

// Input cell read by output cell c at tap (dz, dy, dx): even mirror in z
// (radius one: -1 -> 0, nz -> nz - 1), wrap or valid offset in x and y.
__device__ __forceinline__ int64_t src_cell(const CnnGeom &G, const Cell &c, int dz, int dy,
                                            int dx) {
  int kk = c.k + dz;
  kk = kk < 0 ? 0 : (kk >= G.nz ? G.nz - 1 : kk);
  int jj, ii;
  if (G.periodic) {
    jj = pwrap(c.j + dy, G.nyi);
    ii = pwrap(c.i + dx, G.nxi);
  } else {
    jj = c.j + 1 + dy;
    ii = c.i + 1 + dx;
  }
  return (((int64_t)c.b * G.nz + kk) * G.nyi + jj) * G.nxi + ii;
}

// ------------------------------------------------------------- forward

__global__ __launch_bounds__(kBlock) void pack_kernel(const float *__restrict__ params,
                                                      uint16_t *__restrict__ wbf, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) wbf[q] = f2bf(params[q]);
}

// One thread per (cell, channel) of the channels-last output.
__global__ __launch_bounds__(kBlock) void round_kernel(int64_t n, int C, int64_t cells,
                                                       const float *__restrict__ x,
                                                       const double *__restrict__ scale,
                                                       uint16_t *__restrict__ a0) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * C) return;
  const int c = (int)(q % C);
  const int64_t cell = q / C, b = cell / cells, r = cell - b * cells;
  const float xv = x[(b * C + c) * cells + r];
  const float v = scale ? (float)((double)xv * *scale) : xv;
  a0[q] = f2bf(v);
}

// Layers 1, 2 (16 -> 16) on the matrix cores, as an implicit GEMM per tap:
// D(out ch x 16 cells) += W_tap(out ch x in ch) X_tap(in ch x 16 cells).
// A block owns a 64 x 4 output tile of one batch item and marches up z
// over kCnnKC levels; the input planes k-1, k, k+1 (tile plus a one-cell
// ring, 16 channels, 32 B per cell) sit in a three-plane LDS ring, each
// loaded once with coalesced 16-B loads.  Wave w computes output row w as
// four 16-cell MFMA chains interleaved tap by tap.  Lane l: row = l % 16 is
// its cell (B operand, result) and its output channel (A operand); quad =
// l / 16 selects input channels 4 quad .. 4 quad + 3 (A, B) and output
// channels 4 quad .. 4 quad + 3 of the result.  The 8-B quads of a cell are
// stored at quad ^ ((cell >> 2) & 3) so the 16 lanes reading one quad of 16
// consecutive cells hit distinct LDS banks.
constexpr int kCnnTX = 64, kCnnTY = 4, kCnnKC = 16;
constexpr int kCnnPX = kCnnTX + 2, kCnnPY = kCnnTY + 2;
constexpr int kCnnPlane = kCnnPX * kCnnPY;  // cells per LDS plane

__device__ __forceinline__ int cnn_swz(int cell, int quad) { return quad ^ ((cell >> 2) & 3); }

// Block geometry shared by the tiled layers: a 64 x 4 output tile of batch
// item b over z levels [k0, k1).
struct CnnTile {
  int b, ox0, oy0, ix0, iy0, k0, k1;
};
__device__ __forceinline__ CnnTile cnn_tile(const CnnGeom &G, int tiles_x, int tiles_y,
                                            int chunks) {
  int blk = blockIdx.x;
  CnnTile T;
  const int tx = blk % tiles_x;
  blk /= tiles_x;
  const int ty = blk % tiles_y;
  blk /= tiles_y;
  const int kz = blk % chunks;
  T.b = blk / chunks;
  T.ox0 = tx * kCnnTX;
  T.oy0 = ty * kCnnTY;
  T.ix0 = G.periodic ? T.ox0 - 1 : T.ox0;
  T.iy0 = G.periodic ? T.oy0 - 1 : T.oy0;
  T.k0 = kz * kCnnKC;
  T.k1 = min(G.nz, T.k0 + kCnnKC);
  return T;
}

// Input cell of LDS plane cell (ly, lx): wrap (periodic) or clamp (valid:
// clamped cells feed only masked outputs).
__device__ __forceinline__ int64_t cnn_src(const CnnGeom &G, const CnnTile &T, int kk, int ly,
                                           int lx) {
  kk = kk < 0 ? 0 : (kk >= G.nz ? G.nz - 1 : kk);
  int jj = T.iy0 + ly, ii = T.ix0 + lx;
  if (G.periodic) {
    jj %= G.nyi;
    jj += jj < 0 ? G.nyi : 0;
    ii %= G.nxi;
    ii += ii < 0 ? G.nxi : 0;
  } else {
    jj = jj < G.nyi ? jj : G.nyi - 1;
    ii = ii < G.nxi ? ii : G.nxi - 1;
  }
  return (((int64_t)T.b * G.nz + kk) * G.nyi + jj) * G.nxi + ii;
}

__global__ __launch_bounds__(256) void conv_mid_kernel(CnnGeom G, const uint16_t *__restrict__ ain,
                                                       const float *__restrict__ bias,
                                                       const uint16_t *__restrict__ w,
                                                       float alpha, uint16_t *__restrict__ aout,
                                                       int tiles_x, int tiles_y, int chunks) {
  __shared__ uint2 lds[3][kCnnPlane * 4];  // [slot][cell * 4 + swizzled quad]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, quad = lane >> 4;
  const CnnTile T = cnn_tile(G, tiles_x, tiles_y, chunks);

  bf16x4 wa[kCnnTaps];
#pragma unroll
  for (int t = 0; t < kCnnTaps; ++t)
    wa[t] = *(const bf16x4 *)(w + (t * kCnnCh + row) * kCnnCh + 4 * quad);
  float bq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bq[r] = bias[4 * quad + r];

  // plane kk (mirror-clamped): 2 x 16-B halves per cell, kLoads per thread,
  // fetched into registers first (the next plane's fetch overlaps this
  // plane's products), then stored to a slot
  constexpr int kLoads = (kCnnPlane * 2 + 255) / 256;
  uint4 pre[kLoads];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) {
        const int cell = e >> 1, h = e & 1;
        const int ly = cell / kCnnPX, lx = cell - ly * kCnnPX;
        pre[u] = *(const uint4 *)(ain + cnn_src(G, T, kk, ly, lx) * kCnnCh + 8 * h);
      }
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) {
        const int cell = e >> 1, h = e & 1;
        lds[slot][cell * 4 + cnn_swz(cell, 2 * h)] = make_uint2(pre[u].x, pre[u].y);
        lds[slot][cell * 4 + cnn_swz(cell, 2 * h + 1)] = make_uint2(pre[u].z, pre[u].w);
      }
    }
  };

  fetch(T.k0 - 1);
  store((T.k0 + 2) % 3);
  fetch(T.k0);
  store(T.k0 % 3);
  fetch(T.k0 + 1);
  const int oy = T.oy0 + wv;
  for (int k = T.k0; k < T.k1; ++k) {
    __syncthreads();  // slot (k+1)%3 is no longer read
    store((k + 1) % 3);
    __syncthreads();
    if (k + 1 < T.k1) fetch(k + 2);  // in flight during this level's products
    floatx4 acc[4];
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) acc[t4] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < kCnnTaps; ++t) {
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      const uint2 *plane = lds[(k + dz + 3) % 3];
      const int cbase = (wv + 1 + dy) * kCnnPX + row + 1 + dx;
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int cell = cbase + 16 * t4;
        const uint2 v = plane[cell * 4 + cnn_swz(cell, quad)];
        bf16x4 xb;
        xb[0] = (short)(v.x & 0xFFFFu);
        xb[1] = (short)(v.x >> 16);
        xb[2] = (short)(v.y & 0xFFFFu);
        xb[3] = (short)(v.y >> 16);
        acc[t4] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[t], xb, acc[t4], 0, 0, 0);
      }
    }
    if (oy < G.nyo) {
#pragma unroll
      for (int t4 = 0; t4 < 4; ++t4) {
        const int ox = T.ox0 + 16 * t4 + row;
        if (ox < G.nxo) {
          const uint32_t lo = (uint32_t)f2bf(leaky(acc[t4][0] + bq[0], alpha)) |
                              ((uint32_t)f2bf(leaky(acc[t4][1] + bq[1], alpha)) << 16);
          const uint32_t hi = (uint32_t)f2bf(leaky(acc[t4][2] + bq[2], alpha)) |
                              ((uint32_t)f2bf(leaky(acc[t4][3] + bq[3], alpha)) << 16);
          const int64_t q = (((int64_t)T.b * G.nz + k) * G.nyo + oy) * G.nxo + ox;
          *(uint2 *)(aout + q * kCnnCh + 4 * quad) = make_uint2(lo, hi);
        }
      }
    }
  }
}

// Layer 0 (CI -> 16) on the matrix cores: D(out ch x 16 cells) = W(out ch x
// K) X(K x 16 cells) over the K = 27 CI (tap, channel) pairs, k = tap CI +
// c, padded to a multiple of 16; the im2col operand is gathered from a
// three-plane LDS ring of bfloat16 inputs (channel planes side by side);
// 27 CI / 16 MFMAs (rounded up) per 16 cells.
template <int CI>
__global__ __launch_bounds__(256) void conv_in_kernel(CnnGeom G, const uint16_t *__restrict__ ain,
                                                      const float *__restrict__ params,
                                                      const uint16_t *__restrict__ wbf,
                                                      float alpha, uint16_t *__restrict__ aout,
                                                      int tiles_x, int tiles_y, int chunks) {
  constexpr int K = kCnnTaps * CI, KM = (K + 15) / 16;
  __shared__ uint16_t lds[3][CI][kCnnPlane];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, quad = lane >> 4;
  const CnnTile T = cnn_tile(G, tiles_x, tiles_y, chunks);
  // A operands: W0[tap][o = row][c] for k = 16 m + 4 quad + r
  bf16x4 wa[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = 16 * m + 4 * quad + r;
      wa[m][r] = kk < K ? (short)wbf[((kk / CI) * kCnnCh + row) * CI + kk % CI] : (short)0;
    }
  float bq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bq[r] = params[cnn_bias_offset(CI, 0) + 4 * quad + r];
  // plane kk (mirror-clamped) fetched into registers one plane ahead
  constexpr int kLoads = (kCnnPlane * CI + 255) / 256;
  uint16_t pre[kLoads];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * CI) {
        const int cell = e / CI, c = e - cell * CI;
        const int ly = cell / kCnnPX, lx = cell - ly * kCnnPX;
        pre[u] = ain[cnn_src(G, T, kk, ly, lx) * CI + c];
      }
    }
  };
  auto store = [&](int slot) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * CI) {
        const int cell = e / CI, c = e - cell * CI;
        lds[slot][c][cell] = pre[u];
      }
    }
  };
  fetch(T.k0 - 1);
  store((T.k0 + 2) % 3);
  fetch(T.k0);
  store(T.k0 % 3);
  fetch(T.k0 + 1);
  const int oy = T.oy0 + wv;
  for (int k = T.k0; k < T.k1; ++k) {
    __syncthreads();
    store((k + 1) % 3);
    __syncthreads();
    if (k + 1 < T.k1) fetch(k + 2);
#pragma unroll
    for (int t4 = 0; t4 < 4; ++t4) {
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < KM; ++m) {
        bf16x4 xb;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int kk = 16 * m + 4 * quad + r;
          short v = 0;
          if (kk < K) {
            const int tap = kk / CI, c = kk % CI;
            const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            v = (short)lds[(k + dz + 3) % 3][c][(wv + 1 + dy) * kCnnPX + 16 * t4 + row + 1 + dx];
          }
          xb[r] = v;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[m], xb, acc, 0, 0, 0);
      }
      const int ox = T.ox0 + 16 * t4 + row;
      if (oy < G.nyo && ox < G.nxo) {
        const uint32_t lo = (uint32_t)f2bf(leaky(acc[0] + bq[0], alpha)) |
                            ((uint32_t)f2bf(leaky(acc[1] + bq[1], alpha)) << 16);
        const uint32_t hi = (uint32_t)f2bf(leaky(acc[2] + bq[2], alpha)) |
                            ((uint32_t)f2bf(leaky(acc[3] + bq[3], alpha)) << 16);
        const int64_t q = (((int64_t)T.b * G.nz + k) * G.nyo + oy) * G.nxo + ox;
        *(uint2 *)(aout + q * kCnnCh + 4 * quad) = make_uint2(lo, hi);
      }
    }
  }
}

// Layer 3 (16 -> 1) as a matrix-core product per input plane, then a
// gather.  For every cell of an input plane (the tile plus its one-cell
// ring) D[t][cell] = sum_c W3[t][c] a[cell][c] for the 27 taps t: two
// MFMAs per 16 cells (taps padded to 32 rows of A), kept in LDS.  Output
// cell o then adds, per plane, the D of its 9 neighbours there for the taps
// pointing back at o.  Marching the input planes k0-1 .. k1 (each read as
// its mirror-clamped level, as every layer reads z), plane p completes
// output level p - 1 (planes p - 2, p - 1, p); each thread keeps its output
// cell's three open levels p - 1, p, p + 1 in registers rotated per plane.  LDS bank use: D rows are
// kCnnPlane = 396 floats apart, so the four quads of a wave's D store land
// in disjoint banks; the gather reads consecutive cells per lane.
// GUESS: the output becomes the guess base + s_over_d * y.
template <typename T, bool GUESS>
__global__ __launch_bounds__(256) void conv_out_kernel(CnnGeom G, const uint16_t *__restrict__ ain,
                                                       const float *__restrict__ params,
                                                       const uint16_t *__restrict__ wbf,
                                                       float *__restrict__ y,
                                                       const T *__restrict__ base,
                                                       const double *__restrict__ s_over_d,
                                                       T *__restrict__ guess, int tiles_x,
                                                       int tiles_y, int chunks) {
  __shared__ uint2 lds[kCnnPlane * 4];        // one input plane: 16 channels per cell
  __shared__ float dl[kCnnTaps][kCnnPlane];   // its per-tap products
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, quad = lane >> 4;
  const CnnTile Tl = cnn_tile(G, tiles_x, tiles_y, chunks);
  // A operands: W3[t = 16 m + row][c = 4 quad + r] (one output channel)
  const uint16_t *w3 = wbf + cnn_weight_offset(G.inputs, 3);
  bf16x4 wa[2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 16 * m + row;
      wa[m][r] = t < kCnnTaps ? (short)w3[t * kCnnCh + 4 * quad + r] : (short)0;
    }
  const float b3 = params[cnn_bias_offset(G.inputs, 3)];
  const int lx0 = threadIdx.x & 63, ly0 = threadIdx.x >> 6;  // this thread's output cell
  const int oy = Tl.oy0 + ly0, ox = Tl.ox0 + lx0;
  // plane kk (mirror-clamped) fetched into registers one plane ahead, so
  // the fetch overlaps the previous plane's products and gather
  constexpr int kLoads = (kCnnPlane * 2 + 255) / 256;
  uint4 pre[kLoads];
  auto fetch = [&](int kk) {
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) {
        const int cell = e >> 1, h = e & 1;
        const int ly = cell / kCnnPX, lx = cell - ly * kCnnPX;
        pre[u] = *(const uint4 *)(ain + cnn_src(G, Tl, kk, ly, lx) * kCnnCh + 8 * h);
      }
    }
  };
  float am = 0.f, a0 = 0.f, ap = 0.f;  // output levels p - 1, p, p + 1
  fetch(Tl.k0 - 1);
  for (int p = Tl.k0 - 1; p <= Tl.k1; ++p) {
    __syncthreads();  // the previous plane and its products are no longer read
#pragma unroll
    for (int u = 0; u < kLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) {
        const int cell = e >> 1, h = e & 1;
        lds[cell * 4 + cnn_swz(cell, 2 * h)] = make_uint2(pre[u].x, pre[u].y);
        lds[cell * 4 + cnn_swz(cell, 2 * h + 1)] = make_uint2(pre[u].z, pre[u].w);
      }
    }
    if (p < Tl.k1) fetch(p + 1);
    __syncthreads();
    for (int gi = wv; gi < (kCnnPlane + 15) / 16; gi += 4) {
      const int cell = gi * 16 + row;
      const int cl = cell < kCnnPlane ? cell : kCnnPlane - 1;
      const uint2 v = lds[cl * 4 + cnn_swz(cl, quad)];
      bf16x4 xb;
      xb[0] = (short)(v.x & 0xFFFFu);
      xb[1] = (short)(v.x >> 16);
      xb[2] = (short)(v.y & 0xFFFFu);
      xb[3] = (short)(v.y >> 16);
      const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
      const floatx4 d0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[0], xb, zero, 0, 0, 0);
      const floatx4 d1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[1], xb, zero, 0, 0, 0);
      if (cell < kCnnPlane) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          dl[4 * quad + r][cell] = d0[r];
          if (16 + 4 * quad + r < kCnnTaps) dl[16 + 4 * quad + r][cell] = d1[r];
        }
      }
    }
    __syncthreads();
    // output level p - dz reads plane p at tap row dz
    auto gather = [&](int dz) {
      float sum = 0.f;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
          sum += dl[9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)][(ly0 + 1 + dy) * kCnnPX + lx0 + 1 + dx];
      return sum;
    };
    if (p - 1 >= Tl.k0 && p - 1 < Tl.k1) am += gather(1);
    if (p >= Tl.k0 && p < Tl.k1) a0 += gather(0);
    if (p + 1 >= Tl.k0 && p + 1 < Tl.k1) ap += gather(-1);
    const int oc = p - 1;  // complete now
    if (oc >= Tl.k0 && oc < Tl.k1 && oy < G.nyo && ox < G.nxo) {
      const float out = am + b3;
      const int64_t q = (((int64_t)Tl.b * G.nz + oc) * G.nyo + oy) * G.nxo + ox;
      if (GUESS)
        guess[q] = (T)((double)base[q] + *s_over_d * (double)out);
      else
        y[q] = out;
    }
    am = a0;
    a0 = ap;
    ap = 0.f;
  }
}

// ---------------------------------------------------------------- loss

__device__ __forceinline__ double lh(const float *__restrict__ f, const float *__restrict__ g,
                                     int64_t q, int k, int nz, int64_t sx, int64_t sy,
                                     int64_t plane, double wx, double wy, double wz) {
  // compact Laplacian / d of (f - g) at an interior cell q (g nullable)
  auto e = [&](int64_t p) { return (double)f[p] - (g ? (double)g[p] : 0.0); };
  const int64_t zp = k + 1 < nz ? q + plane : q, zm = k > 0 ? q - plane : q;
  const double c = e(q);
  return wx * (e(q + sx) + e(q - sx) - 2.0 * c) + wy * (e(q + sy) + e(q - sy) - 2.0 * c) +
         wz * (e(zp) + e(zm) - 2.0 * c);
}

__global__ __launch_bounds__(kBlock) void loss_a_kernel(int64_t n, int nz, int ny, int nx,
                                                        double wx, double wy, double wz,
                                                        const float *__restrict__ y,
                                                        const float *__restrict__ t,
                                                        float *__restrict__ qout,
                                                        double *__restrict__ partials) {
  double num = 0.0, den = 0.0;
  const int64_t plane = (int64_t)ny * nx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const Cell c = decode(q, nz, ny, nx);
    float qv = 0.f;
    if (c.j >= 1 && c.j < ny - 1 && c.i >= 1 && c.i < nx - 1) {
      const double qe = lh(y, t, q, c.k, nz, 1, nx, plane, wx, wy, wz);
      const double qt = lh(t, nullptr, q, c.k, nz, 1, nx, plane, wx, wy, wz);
      num += qe * qe;
      den += qt * qt;
      qv = (float)qe;
    }
    qout[q] = qv;
  }
  const double sn = block_sum(num);
  const double sd = block_sum(den);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = sn;
    partials[gridDim.x + blockIdx.x] = sd;
  }
}

__global__ __launch_bounds__(kBlock) void loss_final_kernel(const double *__restrict__ partials,
                                                            int np, double *__restrict__ stats) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    a += partials[q];
    b += partials[np + q];
  }
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    stats[0] = b > 0.0 ? a / b : 0.0;
    stats[1] = b;
    stats[2] = b > 0.0 ? 2.0 / b : 0.0;
  }
}

// gy = (2/den) Lh(q), q zero outside the crop in x and y, mirror in z.
__global__ __launch_bounds__(kBlock) void loss_b_kernel(int64_t n, int nz, int ny, int nx,
                                                        double wx, double wy, double wz,
                                                        const float *__restrict__ qf,
                                                        const double *__restrict__ stats,
                                                        float *__restrict__ gy) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const Cell c = decode(q, nz, ny, nx);
  const int64_t plane = (int64_t)ny * nx;
  const double c0 = qf[q];
  const double xp = c.i + 1 < nx ? qf[q + 1] : 0.0, xm = c.i > 0 ? qf[q - 1] : 0.0;
  const double yp = c.j + 1 < ny ? qf[q + nx] : 0.0, ym = c.j > 0 ? qf[q - nx] : 0.0;
  const double zp = qf[c.k + 1 < nz ? q + plane : q], zm = qf[c.k > 0 ? q - plane : q];
  const double v = wx * (xp + xm) + wy * (yp + ym) + wz * (zp + zm) - 2.0 * (wx + wy + wz) * c0;
  gy[q] = (float)(stats[2] * v);
}

// ------------------------------------------------------------ backward

// gprev(cell', i) = leaky'(ain(cell', i)) * sum over (tap, out cell, o) with
// src(out cell, tap) = cell' of gy(out cell, o) W[tap][o][i].  The z mirror
// makes wall cells receive a second term: out level 0 at dz = -1 reads
// level 0, out level nz-1 at dz = +1 reads level nz-1.
template <int CI, int CO>
__global__ __launch_bounds__(kBlock) void dgrad_kernel(CnnGeom G, const float *__restrict__ gy,
                                                       const uint16_t *__restrict__ wl,
                                                       const uint16_t *__restrict__ ain,
                                                       float alpha, float *__restrict__ gprev) {
  __shared__ float w[kCnnTaps * CO * CI];
  for (int e = threadIdx.x; e < kCnnTaps * CO * CI; e += blockDim.x) w[e] = bf2f(wl[e]);
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= G.n_in) return;
  const Cell c = decode(q, G.nz, G.nyi, G.nxi);
  float acc[CI];
#pragma unroll
  for (int i = 0; i < CI; ++i) acc[i] = 0.f;
  for (int dz = -1; dz <= 1; ++dz) {
    int ks[2], nk = 0;
    if (c.k - dz >= 0 && c.k - dz < G.nz) ks[nk++] = c.k - dz;
    if ((dz == -1 && c.k == 0) || (dz == 1 && c.k == G.nz - 1)) ks[nk++] = c.k;
    for (int dy = -1; dy <= 1; ++dy) {
      const int j = c.j - 1 - dy;
      if (j < 0 || j >= G.nyo) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int i = c.i - 1 - dx;
        if (i < 0 || i >= G.nxo) continue;
        const int t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
        for (int m = 0; m < nk; ++m) {
          const float *g = gy + ((((int64_t)c.b * G.nz + ks[m]) * G.nyo + j) * G.nxo + i) * CO;
#pragma unroll 2
          for (int o = 0; o < CO; ++o) {
            const float gv = g[o];
            const float *wr = w + (t * CO + o) * CI;
#pragma unroll
            for (int i2 = 0; i2 < CI; ++i2) acc[i2] += gv * wr[i2];
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const bool neg = (ain[q * CI + i] & 0x8000u) != 0;
    gprev[q * CI + i] = acc[i] * (neg ? alpha : 1.f);
  }
}

// Weight gradient partials of one block of `chunk` output cells: thread
// pair (o, i) accumulates the 27 taps in FP64 (products of an FP32 gradient
// and a bfloat16 activation are exact in FP64); PAIRS < 256 spreads the
// cells over 256 / PAIRS groups, summed in a fixed order through LDS.
// Partials layout per block: [tap][o][i] then the CO bias entries.
template <int CI, int CO>
__global__ __launch_bounds__(kBlock) void wgrad_kernel(CnnGeom G, const float *__restrict__ gy,
                                                       const uint16_t *__restrict__ ain,
                                                       int64_t chunk, double *__restrict__ partials) {
  constexpr int PAIRS = CI * CO;
  constexpr int GROUPS = kBlock / PAIRS;
  constexpr int E = kCnnTaps * PAIRS + CO;
  __shared__ double red[kBlock];
  const int pair = threadIdx.x % PAIRS, grp = threadIdx.x / PAIRS;
  const int o = pair / CI, ci = pair % CI;
  double acc[kCnnTaps + 1];
#pragma unroll
  for (int t = 0; t <= kCnnTaps; ++t) acc[t] = 0.0;
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = c0 + chunk < G.n_out ? c0 + chunk : G.n_out;
  // threads beyond GROUPS * PAIRS (PAIRS not dividing the block) stay idle
  for (int64_t q = c0 + grp; grp < GROUPS && q < c1; q += GROUPS) {
    const Cell c = decode(q, G.nz, G.nyo, G.nxo);
    const double g = gy[q * CO + o];
    acc[kCnnTaps] += g;
#pragma unroll
    for (int t = 0; t < kCnnTaps; ++t) {
      const int64_t src = src_cell(G, c, t / 9 - 1, (t / 3) % 3 - 1, t % 3 - 1);
      acc[t] += g * (double)bf2f(ain[src * CI + ci]);
    }
  }
  double *out = partials + (int64_t)blockIdx.x * E;
  for (int t = 0; t <= kCnnTaps; ++t) {
    double v = acc[t];
    if (GROUPS > 1) {
      __syncthreads();
      red[threadIdx.x] = v;
      __syncthreads();
      if (grp == 0)
        for (int m = 1; m < GROUPS; ++m) v += red[m * PAIRS + pair];
    }
    if (grp == 0) {
      if (t < kCnnTaps)
        out[t * PAIRS + pair] = v;
      else if (ci == 0)
        out[kCnnTaps * PAIRS + o] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void wgrad_final_kernel(const double *__restrict__ partials,
                                                             int nblocks, int E, int nw,
                                                             float *__restrict__ gw,
                                                             float *__restrict__ gb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * E + e];
  if (e < nw)
    gw[e] = (float)s;
  else
    gb[e - nw] = (float)s;
}

__global__ __launch_bounds__(kBlock) void adam_kernel(int n, float *__restrict__ p,
                                                      const float *__restrict__ g,
                                                      float *__restrict__ m, float *__restrict__ v,
                                                      float lr, float b1, float b2, float omb1,
                                                      float omb2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + omb1 * gq;
  const float vq = b2 * v[q] + omb2 * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// ------------------------------------------------- inputs and datasets

template <typename T>
__global__ __launch_bounds__(kBlock) void residual_kernel(Grid g, double ix2, double iy2,
                                                          double iz2, const T *__restrict__ rhs,
                                                          const T *__restrict__ base,
                                                          float *__restrict__ r,
                                                          double *__restrict__ partials) {
  double acc = 0.0;
  // block b takes the x rows b, b + gridDim.x, ... (level and y index uniform)
  const int64_t rows = (int64_t)g.ny * g.nz;
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const int k = (int)(row / g.ny), j = (int)(row - (int64_t)k * g.ny);
    const T *c0 = base ? base + row * g.nx : nullptr;
    const T *yp = base ? base + ((int64_t)k * g.ny + pwrap(j + 1, g.ny)) * g.nx : nullptr;
    const T *ym = base ? base + ((int64_t)k * g.ny + pwrap(j - 1, g.ny)) * g.nx : nullptr;
    const T *zp = base ? base + ((int64_t)zmirror(k + 1, g.nz) * g.ny + j) * g.nx : nullptr;
    const T *zm = base ? base + ((int64_t)zmirror(k - 1, g.nz) * g.ny + j) * g.nx : nullptr;
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
      const int64_t q = row * g.nx + i;
      double v = (double)rhs[q];
      if (base) {
        const int ip = i + 1 < g.nx ? i + 1 : 0, im = i > 0 ? i - 1 : g.nx - 1;
        const double c = c0[i];
        const double lap = ((double)c0[ip] + (double)c0[im] - 2.0 * c) * ix2 +
                           ((double)yp[i] + (double)ym[i] - 2.0 * c) * iy2 +
                           ((double)zp[i] + (double)zm[i] - 2.0 * c) * iz2;
        v -= lap;
      }
      r[q] = (float)v;
      acc += v * v;
    }
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void scale_kernel(const double *__restrict__ partials, int np,
                                                       double n, double d, double *__restrict__ sc) {
  double a = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) a += partials[q];
  a = block_sum(a);
  if (threadIdx.x == 0) {
    const double s = sqrt(a / n);
    sc[0] = s;
    sc[1] = s > 0.0 ? 1.0 / s : 0.0;
    sc[2] = s / d;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void pair_kernel(int64_t n, const float *__restrict__ r,
                                                      const T *__restrict__ phi,
                                                      const T *__restrict__ base,
                                                      const double *__restrict__ sc, double d,
                                                      float *__restrict__ x, float *__restrict__ t) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double inv = sc[1];
  x[q] = (float)((double)r[q] * inv);
  t[q] = (float)(((double)phi[q] - (base ? (double)base[q] : 0.0)) * d * inv);
}

// Three-input network inputs at cell q: (r/s, base d/s, rhs/s), FP64
// products rounded once.
template <typename T>
__device__ __forceinline__ void inputs3(int64_t q, const float *__restrict__ r,
                                        const T *__restrict__ base, const T *__restrict__ rhs,
                                        double inv, double d, float v[3]) {
  v[0] = (float)((double)r[q] * inv);
  v[1] = (float)((double)base[q] * d * inv);
  v[2] = (float)((double)rhs[q] * inv);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void input3_kernel(int64_t n, const float *__restrict__ r,
                                                        const T *__restrict__ base,
                                                        const T *__restrict__ rhs,
                                                        const double *__restrict__ sc, double d,
                                                        uint16_t *__restrict__ a0) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  float v[3];
  inputs3(q, r, base, rhs, sc[1], d, v);
  a0[3 * q] = f2bf(v[0]);
  a0[3 * q + 1] = f2bf(v[1]);
  a0[3 * q + 2] = f2bf(v[2]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void pair3_kernel(int64_t n, const float *__restrict__ r,
                                                       const T *__restrict__ base,
                                                       const T *__restrict__ rhs,
                                                       const T *__restrict__ phi,
                                                       const double *__restrict__ sc, double d,
                                                       float *__restrict__ x,
                                                       float *__restrict__ t) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double inv = sc[1];
  float v[3];
  inputs3(q, r, base, rhs, inv, d, v);
  x[q] = v[0];
  x[n + q] = v[1];
  x[2 * n + q] = v[2];
  if (phi) t[q] = (float)(((double)phi[q] - (double)base[q]) * d * inv);
}

// Stored layer input (channels-last bfloat16, C channels, `cells` cells per
// batch entry) to FP32 in (batch, C, cells) order.
__global__ __launch_bounds__(kBlock) void unpack_kernel(int64_t n, int C, int64_t cells,
                                                        const uint16_t *__restrict__ a,
                                                        float *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // input order
  if (q >= n) return;
  const int c = (int)(q % C);
  const int64_t cell = q / C;
  const int64_t b = cell / cells, r = cell - b * cells;
  out[(b * C + c) * cells + r] = bf2f(a[q]);
}

// As pair_kernel with the residual r already in x: x = x/s in place.
template <typename T>
__global__ __launch_bounds__(kBlock) void pair_inplace_kernel(int64_t n, const T *__restrict__ phi,
                                                              const T *__restrict__ base,
                                                              const double *__restrict__ sc,
                                                              double d, float *x,
                                                              float *__restrict__ t) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double inv = sc[1];
  x[q] = (float)((double)x[q] * inv);
  t[q] = (float)(((double)phi[q] - (base ? (double)base[q] : 0.0)) * d * inv);
}

// Input crops (batch, C, nz, cy + 8, cx + 8) read as C nz levels per item
// (channel-major, so level index c nz + k); targets (batch, nz, cy, cx).
__global__ __launch_bounds__(kBlock) void gather_kernel(const float *__restrict__ X,
                                                        const float *__restrict__ Tt,
                                                        int64_t field, int C, int nz, int ny,
                                                        int nx, const int32_t *__restrict__ crops,
                                                        int npairs, int cy, int cx, int64_t n_in,
                                                        int64_t n_t,
                                                        float *__restrict__ xb,
                                                        float *__restrict__ tb) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool is_x = q < n_in;
  if (q >= n_in + n_t) return;
  const int64_t qq = is_x ? q : q - n_in;
  const int h = is_x ? 4 : 0;
  const int lv = is_x ? C * nz : nz;  // levels per item
  const Cell c = decode(qq, lv, cy + 2 * h, cx + 2 * h);
  // every index is reduced modulo its range, so any crop entry reads in bounds
  const int32_t *cr = crops + 3 * c.b;
  int p = cr[0] % npairs, j = (int)(((int64_t)cr[1] - h + c.j) % ny),
      i = (int)(((int64_t)cr[2] - h + c.i) % nx);
  p += p < 0 ? npairs : 0;
  j += j < 0 ? ny : 0;
  i += i < 0 ? nx : 0;
  const int64_t stride = is_x ? field * C : field;  // one pair
  const int64_t src = (int64_t)p * stride + ((int64_t)c.k * ny + j) * nx + i;
  if (is_x)
    xb[qq] = X[src];
  else
    tb[qq] = Tt[src];
}

}  // namespace

// ----------------------------------------------------------- launchers

void launch_cnn_pack(const float *params, int n, uint16_t *wbf, hipStream_t s) {
  pack_kernel<<<blocks_for(n), kBlock, 0, s>>>(params, wbf, n);
}

void launch_cnn_round(int64_t n, int C, int64_t cells, const float *x, const double *scale,
                      uint16_t *a0, hipStream_t s) {
  round_kernel<<<blocks_for(n * C), kBlock, 0, s>>>(n, C, cells, x, scale, a0);
}

void launch_cnn_conv(int layer, const CnnGeom &G, const uint16_t *ain, const float *params,
                     const uint16_t *wbf, float alpha, uint16_t *aout, float *yout, hipStream_t s) {
  const int tiles_x = (G.nxo + kCnnTX - 1) / kCnnTX, tiles_y = (G.nyo + kCnnTY - 1) / kCnnTY;
  const int chunks = (G.nz + kCnnKC - 1) / kCnnKC;
  const unsigned blocks = (unsigned)((int64_t)G.batch * tiles_x * tiles_y * chunks);
  if (layer == 0) {
    if (G.inputs == 3)
      conv_in_kernel<3><<<blocks, 256, 0, s>>>(G, ain, params, wbf, alpha, aout, tiles_x, tiles_y,
                                               chunks);
    else
      conv_in_kernel<1><<<blocks, 256, 0, s>>>(G, ain, params, wbf, alpha, aout, tiles_x, tiles_y,
                                               chunks);
  } else if (layer < kCnnLayers - 1) {
    conv_mid_kernel<<<blocks, 256, 0, s>>>(G, ain, params + cnn_bias_offset(G.inputs, layer),
                                           wbf + cnn_weight_offset(G.inputs, layer), alpha, aout,
                                           tiles_x, tiles_y, chunks);
  } else {
    conv_out_kernel<float, false><<<blocks, 256, 0, s>>>(G, ain, params, wbf, yout, nullptr,
                                                         nullptr, nullptr, tiles_x, tiles_y,
                                                         chunks);
  }
}

template <typename T>
void launch_cnn_guess(const CnnGeom &G, const uint16_t *ain, const float *params,
                      const uint16_t *wbf, const T *base, const double *s_over_d, T *guess,
                      hipStream_t s) {
  const int tiles_x = (G.nxo + kCnnTX - 1) / kCnnTX, tiles_y = (G.nyo + kCnnTY - 1) / kCnnTY;
  const int chunks = (G.nz + kCnnKC - 1) / kCnnKC;
  const unsigned blocks = (unsigned)((int64_t)G.batch * tiles_x * tiles_y * chunks);
  conv_out_kernel<T, true><<<blocks, 256, 0, s>>>(G, ain, params, wbf, nullptr, base, s_over_d,
                                                  guess, tiles_x, tiles_y, chunks);
}

void launch_cnn_loss(int batch, int nz, int ny, int nx, double wx, double wy, double wz,
                     const float *y, const float *t, float *q, double *partials, double *stats,
                     float *gy, hipStream_t s) {
  const int64_t n = (int64_t)batch * nz * ny * nx;
  loss_a_kernel<<<kReduceBlocks, kBlock, 0, s>>>(n, nz, ny, nx, wx, wy, wz, y, t, q, partials);
  loss_final_kernel<<<1, kBlock, 0, s>>>(partials, kReduceBlocks, stats);
  if (gy) loss_b_kernel<<<blocks_for(n), kBlock, 0, s>>>(n, nz, ny, nx, wx, wy, wz, q, stats, gy);
}

void launch_cnn_dgrad(int layer, const CnnGeom &G, const float *gy, const uint16_t *wbf,
                      const uint16_t *ain, float alpha, float *gprev, hipStream_t s) {
  const uint16_t *wl = wbf + cnn_weight_offset(G.inputs, layer);
  if (layer == kCnnLayers - 1)
    dgrad_kernel<kCnnCh, 1><<<blocks_for(G.n_in), kBlock, 0, s>>>(G, gy, wl, ain, alpha, gprev);
  else
    dgrad_kernel<kCnnCh, kCnnCh><<<blocks_for(G.n_in), kBlock, 0, s>>>(G, gy, wl, ain, alpha,
                                                                        gprev);
}

void launch_cnn_wgrad(int layer, const CnnGeom &G, const float *gy, const uint16_t *ain,
                      double *partials, float *grad, hipStream_t s) {
  const int ci = cnn_cin(G.inputs, layer), co = cnn_cout(layer);
  const int E = kCnnTaps * ci * co + co;
  const int64_t chunk = (G.n_out + kCnnWgradBlocks - 1) / kCnnWgradBlocks;
  if (ci == 1)
    wgrad_kernel<1, kCnnCh><<<kCnnWgradBlocks, kBlock, 0, s>>>(G, gy, ain, chunk, partials);
  else if (ci == 3)
    wgrad_kernel<3, kCnnCh><<<kCnnWgradBlocks, kBlock, 0, s>>>(G, gy, ain, chunk, partials);
  else if (co == 1)
    wgrad_kernel<kCnnCh, 1><<<kCnnWgradBlocks, kBlock, 0, s>>>(G, gy, ain, chunk, partials);
  else
    wgrad_kernel<kCnnCh, kCnnCh><<<kCnnWgradBlocks, kBlock, 0, s>>>(G, gy, ain, chunk, partials);
  wgrad_final_kernel<<<blocks_for(E), kBlock, 0, s>>>(partials, kCnnWgradBlocks, E,
                                                      kCnnTaps * ci * co,
                                                      grad + cnn_weight_offset(G.inputs, layer),
                                                      grad + cnn_bias_offset(G.inputs, layer));
}

void launch_cnn_adam(int n, float *params, const float *grad, float *m, float *v, int step,
                     double lr, double beta1, double beta2, double eps, hipStream_t s) {
  const double c1 = 1.0 - std::pow(beta1, step), c2 = 1.0 - std::pow(beta2, step);
  // 1 - beta in FP64: 1.f - 0.999f carries a 5e-5 relative error
  adam_kernel<<<blocks_for(n), kBlock, 0, s>>>(n, params, grad, m, v, (float)lr, (float)beta1,
                                               (float)beta2, (float)(1.0 - beta1),
                                               (float)(1.0 - beta2), (float)eps, (float)c1,
                                               (float)c2);
}

template <typename T>
void launch_cnn_residual(const Grid &g, const T *rhs, const T *base, float *r, double *partials,
                         hipStream_t s) {
  residual_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(g, 1.0 / (g.dx * g.dx), 1.0 / (g.dy * g.dy),
                                                      1.0 / (g.dz * g.dz), rhs, base, r, partials);
}

void launch_cnn_scale(const double *partials, double n, double d, double *sc, hipStream_t s) {
  scale_kernel<<<1, kBlock, 0, s>>>(partials, kReduceBlocks, n, d, sc);
}

template <typename T>
void launch_cnn_pair(const Grid &g, const float *r, const T *phi, const T *base, const double *sc,
                     double d, float *x, float *t, hipStream_t s) {
  pair_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, r, phi, base, sc, d, x, t);
}

template <typename T>
void launch_cnn_input3(const Grid &g, const float *r, const T *base, const T *rhs,
                       const double *sc, double d, uint16_t *a0, hipStream_t s) {
  input3_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, r, base, rhs, sc, d, a0);
}

template <typename T>
void launch_cnn_pair3(const Grid &g, const float *r, const T *base, const T *rhs, const T *phi,
                      const double *sc, double d, float *x, float *t, hipStream_t s) {
  pair3_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, r, base, rhs, phi, sc, d, x, t);
}

void launch_cnn_unpack(const CnnGeom &G, int C, const uint16_t *a, float *out, hipStream_t s) {
  const int64_t n = G.n_in * C;
  unpack_kernel<<<blocks_for(n), kBlock, 0, s>>>(n, C, (int64_t)G.nz * G.nyi * G.nxi, a, out);
}

template <typename T>
void launch_cnn_pair_inplace(const Grid &g, const T *phi, const T *base, const double *sc,
                             double d, float *x, float *t, hipStream_t s) {
  pair_inplace_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, phi, base, sc, d, x, t);
}

void launch_cnn_gather(const float *X, const float *Tt, int npairs, int C, int nz, int ny, int nx,
                       const int32_t *crops, int batch, int cy, int cx, float *xb, float *tb,
                       hipStream_t s) {
  const int64_t n_in = (int64_t)batch * C * nz * (cy + 8) * (cx + 8);
  const int64_t n_t = (int64_t)batch * nz * cy * cx;
  gather_kernel<<<blocks_for(n_in + n_t), kBlock, 0, s>>>(X, Tt, (int64_t)nz * ny * nx, C, nz, ny,
                                                          nx, crops, npairs, cy, cx, n_in, n_t,
                                                          xb, tb);
}

#define CNN_INST(T)                                                                             \
  template void launch_cnn_guess<T>(const CnnGeom &, const uint16_t *, const float *,            \
                                    const uint16_t *, const T *, const double *, T *,            \
                                    hipStream_t);                                                \
  template void launch_cnn_residual<T>(const Grid &, const T *, const T *, float *, double *,   \
                                       hipStream_t);                                             \
  template void launch_cnn_pair<T>(const Grid &, const float *, const T *, const T *,            \
                                   const double *, double, float *, float *, hipStream_t);        \
  template void launch_cnn_pair_inplace<T>(const Grid &, const T *, const T *, const double *,   \
                                           double, float *, float *, hipStream_t);              \
  template void launch_cnn_input3<T>(const Grid &, const float *, const T *, const T *,          \
                                     const double *, double, uint16_t *, hipStream_t);           \
  template void launch_cnn_pair3<T>(const Grid &, const float *, const T *, const T *, const T *, \
                                    const double *, double, float *, float *, hipStream_t);
CNN_INST(float)
CNN_INST(double)
#undef CNN_INST

}  // namespace lesmi
