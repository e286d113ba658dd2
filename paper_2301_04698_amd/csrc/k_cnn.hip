// Guess network kernels: inference of the learned Poisson initial guess and
// the forward/backward/update kernels that train it on solver-generated
// pairs.
//
// Layouts: single-channel fields are (batch, nz, ny, nx) with x fastest;
// network inputs of C channels are (batch, C, nz, ny, nx) in FP32 and
// channels-last bfloat16 (cell * C + c) once rounded; 16-channel
// activations are channels-last bfloat16 (cell * 16 + c), so one cell's
// channels are one 32-byte line.  Inference runs on the matrix cores with
// FP32 accumulation: the 16 -> 16 and 16 -> 1 layers as implicit GEMMs
// over pairs of in-plane taps (16 consecutive output cells per product),
// the C -> 16 layer as one GEMM over (tap, channel) pairs.  The backward
// pass is FP32 vector code (FP64 sums in the weight gradient).
#include <cmath>
#include <type_traits>

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

// FP32 -> bfloat16, round to nearest, ties to even: the conversion
// instruction of gfx950 (v_cvt_pk_bf16_f32, two values per instruction).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
// bf16(a) in the low half, bf16(b) in the high half.
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2_t{a, b}, bf16x2_t));
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

// Layers 1, 2 (16 -> 16) and 3 (16 -> 1) on the matrix cores as implicit
// GEMMs over pairs of in-plane taps (K = 32: two taps x 16 input channels).
// A block owns a 64 x 4 output tile of one batch item and marches the input
// planes k0 - 1 .. k1 of its z chunk [k0, k1) (each read as its
// mirror-clamped level, as every layer reads z).  Input plane p feeds
// output levels p + 1, p and p - 1 through the tap rows dz = -1, 0, +1, so
// each operand read from LDS serves three products and level p - 1 is
// complete once plane p is done.  A plane (the tile plus a one-cell ring,
// 16 channels, 32 B per cell) is loaded once with coalesced 16-B loads into
// one slot of a two-slot LDS ring while the other slot is read, one
// barrier per plane.  Wave w computes output row w as four 16-cell chains.
constexpr int kCnnTX = 64, kCnnTY = 4, kCnnKC = 16;
constexpr int kCnnPX = kCnnTX + 2, kCnnPY = kCnnTY + 2;
constexpr int kCnnPlane = kCnnPX * kCnnPY;  // cells per LDS plane
// In-plane tap pairs: pair m joins the taps 2m and 2m + 1 of the 3 x 3
// plane stencil (t = 3 (dy + 1) + (dx + 1)); the second tap of pair 4 has
// zero weights and reads tap 8 again.
constexpr int kCnnPairs = 5;
// LDS cell stride: the two 16-B channel halves, unpadded.  Measured on
// gfx950, 16-B operand reads of this layout (lanes l % 16 on consecutive
// cells, the two halves on alternate lane groups) run at the rate of fully
// contiguous reads, while a 48-B stride costs 1.8x.
constexpr int kCnnCellB = 32;

// Block geometry shared by the tiled layers: a 64 x 4 output tile of batch
// item b over z levels [k0, k1).  The grid is a multiple of 8 blocks and
// XCD x (the blocks b with b % 8 = x) takes the x-th contiguous range of
// tiles in the order x tile, y tile, z chunk, batch item, so that tiles
// next to each other in y run on one XCD and share their halo rows in its
// L2.  Blocks past the last tile are not valid.
struct CnnTile {
  int b, ox0, oy0, ix0, iy0, k0, k1;
  bool valid;
};
inline unsigned cnn_blocks(int64_t tiles) { return (unsigned)((tiles + 7) / 8 * 8); }
__device__ __forceinline__ CnnTile cnn_tile(const CnnGeom &G, int tiles_x, int tiles_y,
                                            int chunks) {
  const int per = (int)(gridDim.x >> 3);
  int blk = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  CnnTile T;
  T.valid = blk < G.batch * tiles_x * tiles_y * chunks;
  if (!T.valid) blk = 0;
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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight bfloat16 weights w[0..7] (8-B aligned) as one K = 32 operand half.
__device__ __forceinline__ bf16x8 load_w8(const uint16_t *__restrict__ w) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 lo = *(const u32x2 *)w, hi = *(const u32x2 *)(w + 4);
  return __builtin_bit_cast(bf16x8, u32x4{lo.x, lo.y, hi.x, hi.y});
}

// Operand register layout of a K = 32 product (v_mfma_f32_16x16x32_bf16):
// lane l holds row / column l % 16 and k = 8 (l / 16) .. 8 (l / 16) + 7,
// i.e. side = l / 32 picks the tap of the pair and half = (l / 16) % 2 the
// input channels 8 half .. 8 half + 7.  The activation operand of lane l
// is cell l % 16 of its chain, shifted by its tap: the byte offset of that
// cell's channel half within an LDS plane, for pair m and chain 0 of wave
// wv (chain c adds 16 c cells).
__device__ __forceinline__ uint32_t pair_offset(int wv, int row, int side, int half, int m) {
  const int t = min(2 * m + side, 8);
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  return (uint32_t)(((wv + 1 + dy) * kCnnPX + row + 1 + dx) * kCnnCellB + 16 * half);
}

// Plane streaming of the tiled 16-channel layers: 2 x 16-B halves per cell
// of the plane (tile plus ring), kPlaneLoads per thread.  The in-plane
// source cell of each load (wrap or clamp) is fixed per thread; a plane
// adds its level's offset.
constexpr int kPlaneLoads = (kCnnPlane * 2 + 255) / 256;

__device__ __forceinline__ void plane_sources(const CnnGeom &G, const CnnTile &T,
                                              int32_t (&src)[kPlaneLoads]) {
#pragma unroll
  for (int u = 0; u < kPlaneLoads; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int cell = min(e >> 1, kCnnPlane - 1);
    const int ly = cell / kCnnPX, lx = cell - ly * kCnnPX;
    // in-plane part of cnn_src: level 0 of batch item 0
    const CnnTile T0 = {0, T.ox0, T.oy0, T.ix0, T.iy0, 0, 0, true};
    src[u] = (int32_t)cnn_src(G, T0, 0, ly, lx) * kCnnCh + 8 * (e & 1);
  }
}

// Element offset of level kk (mirror-clamped) of batch item b.
__device__ __forceinline__ int64_t plane_base(const CnnGeom &G, int b, int kk) {
  kk = kk < 0 ? 0 : (kk >= G.nz ? G.nz - 1 : kk);
  return ((int64_t)b * G.nz + kk) * G.nyi * G.nxi * kCnnCh;
}

// Layers 1, 2: aout = bf16(leaky(conv(ain) + b)).  Lane l: row = l % 16 is
// its output channel in the weight operand and its cell in the activation
// operand and the result, which holds output channels 4 (l / 16) .. + 3.
// FUSED (inference of the one-input network on a periodic field): layer 0
// runs inside the block.  Each plane of layer 0's output is computed on
// the tile plus its ring (bias, leaky ReLU, bfloat16) straight into the
// LDS slot that layer 1 reads, from the network input: the FP32 residual r
// times *in_scale, rounded to bfloat16 as the separate input pass does.
// The input levels (the tile plus a two-cell ring) are staged once each in
// a four-slot LDS ring: layer-0 plane P reads levels c - 1, c, c + 1 of c =
// P clamped to the grid (each again clamped; virtual level u sits in slot
// (u + 4) mod 4), and each plane step stages the one level the next plane
// adds.  Layer 0's activations never reach HBM.
constexpr int kInPX = kCnnPX + 2, kInPY = kCnnPY + 2;
constexpr int kInPlane = kInPX * kInPY;           // input cells per plane
constexpr int kInLoads = (kInPlane + 255) / 256;  // per thread and level
constexpr int kL0Chains = (kCnnPlane + 15) / 16;

typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

template <bool FUSED>
__global__ __launch_bounds__(256, 2) void conv_mid_kernel(
    CnnGeom G, const uint16_t *__restrict__ ain, const float *__restrict__ rin,
    const double *__restrict__ in_scale, const float *__restrict__ bias0,
    const uint16_t *__restrict__ w0, const float *__restrict__ bias,
    const uint16_t *__restrict__ w, float alpha, uint16_t *__restrict__ aout, int tiles_x,
    int tiles_y, int chunks) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][kCnnPlane * kCnnCellB];
  // fused: the ring of staged input levels, one bfloat16 value per 32-bit
  // word so that every operand read is an aligned word
  __shared__ uint32_t inr[FUSED ? 4 : 1][FUSED ? kInPlane : 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, quad = lane >> 4, side = quad >> 1, half = quad & 1;
  const CnnTile T = cnn_tile(G, tiles_x, tiles_y, chunks);
  if (!T.valid) return;  // the whole block
  auto slot = [&](int p) { return (p - T.k0 + 1) & 1; };  // LDS slot of plane p

  // weights W[9 (dz + 1) + t][o = row][8 half .. + 7], t = 2 m + side
  bf16x8 wa[3][kCnnPairs];
  uint32_t poff[kCnnPairs];
#pragma unroll
  for (int m = 0; m < kCnnPairs; ++m) {
    const int t = 2 * m + side;
#pragma unroll
    for (int z = 0; z < 3; ++z)
      wa[z][m] = t < 9 ? load_w8(w + ((9 * z + t) * kCnnCh + row) * kCnnCh + 8 * half)
                       : bf16x8{};
    poff[m] = pair_offset(wv, row, side, half, m);
  }
  float bq[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bq[r] = bias[4 * quad + r];
  const int oy = T.oy0 + wv;

  // ---- how a plane reaches its LDS slot
  // (a) layer-1 input from HBM: plane kk fetched into registers one plane
  // ahead (the loads past the plane repeat its last cell and are not
  // stored), then stored to a slot
  int32_t src[FUSED ? 1 : kPlaneLoads];
  u32x4 pre[FUSED ? 1 : kPlaneLoads];
  // (b) fused layer 0: the one input level a plane step adds to the ring,
  // fetched a step ahead as FP32 and rounded when stored
  int32_t gof[FUSED ? kInLoads : 1];
  float rpre[FUSED ? kInLoads : 1];
  bf16x8 w0a[2];
  float b0q[4];
  double scale = 0.0;
  if constexpr (FUSED) {
#pragma unroll
    for (int u = 0; u < kInLoads; ++u) {
      const int cell = min((int)threadIdx.x + 256 * u, kInPlane - 1);
      const int iy = cell / kInPX, ix = cell - iy * kInPX;
      const int jj = pwrap(T.oy0 - 2 + iy, G.nyi), ii = pwrap(T.ox0 - 2 + ix, G.nxi);
      gof[u] = jj * G.nxi + ii;
    }
    // layer-0 weight operand: k = 8 quad + e of product m is tap 9 quad +
    // (8 m + e) (dz = quad - 1; in-plane taps 0..8), zero past them
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      u16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int cb = 8 * m + e;
        v[e] = quad < 3 && cb < 9 ? w0[(9 * quad + cb) * kCnnCh + row] : (uint16_t)0;
      }
      w0a[m] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) b0q[r] = bias0[4 * quad + r];
    scale = *in_scale;
  } else {
    plane_sources(G, T, src);
  }
  const int64_t in_plane = (int64_t)G.nyi * G.nxi;
  auto clampz = [&](int P) { return P < 0 ? 0 : (P >= G.nz ? G.nz - 1 : P); };
  // virtual input level u (content: level u clamped) into registers, then
  // into ring slot (u + 4) mod 4
  auto fetch_level = [&](int u) __attribute__((always_inline)) {
    const int64_t base = ((int64_t)T.b * G.nz + clampz(u)) * in_plane;
#pragma unroll
    for (int i = 0; i < kInLoads; ++i) rpre[i] = rin[base + gof[i]];
  };
  auto store_level = [&](int u) __attribute__((always_inline)) {
    uint32_t *dst = inr[(u + 4) & 3];
#pragma unroll
    for (int i = 0; i < kInLoads; ++i) {
      const int e = (int)threadIdx.x + 256 * i;
      if (e < kInPlane) dst[e] = f2bf((float)((double)rpre[i] * scale));
    }
  };
  // chain k of layer-0 plane P (its three input levels in the ring) into
  // slot(P): wave w takes the 16-cell chains w + 4 k, k = 0..6, of the
  // tile-plus-ring plane (k = 6 only for wave 0: 25 chains)
  auto layer0_chain = [&](int k, int P) __attribute__((always_inline)) {
    const uint32_t *in = inr[(clampz(P) - 1 + min(quad, 2) + 4) & 3];
    unsigned char *dst = lds[slot(P)];
    {
      const int ch = wv + 4 * k;
      const int cell = ch * 16 + row, cc = min(cell, kCnnPlane - 1);
      const int ay = cc / kCnnPX, ax = cc - ay * kCnnPX;
      const uint32_t *pl = in + (ay + 1) * kInPX + ax + 1;
      u16x8 v0, v1 = {};
#pragma unroll
      for (int e = 0; e < 8; ++e) v0[e] = (uint16_t)pl[(e / 3 - 1) * kInPX + (e % 3 - 1)];
      v1[0] = (uint16_t)pl[kInPX + 1];  // in-plane tap 8
      floatx4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma32(w0a[0], __builtin_bit_cast(bf16x8, v0), acc);
      acc = mfma32(w0a[1], __builtin_bit_cast(bf16x8, v1), acc);
      if (cell < kCnnPlane) {
        const uint32_t l2 = f2bf2(leaky(acc[0] + b0q[0], alpha),
                                  leaky(acc[1] + b0q[1], alpha));
        const uint32_t h2 = f2bf2(leaky(acc[2] + b0q[2], alpha),
                                  leaky(acc[3] + b0q[3], alpha));
        *(uint2 *)(dst + cell * kCnnCellB + 8 * quad) = make_uint2(l2, h2);
      }
    }
  };
  auto layer0 = [&](int P) __attribute__((always_inline)) {
#pragma unroll
    for (int k = 0; k < 6; ++k) layer0_chain(k, P);
    if (wv == 0) layer0_chain(6, P);
  };
  auto fetch = [&](int kk) __attribute__((always_inline)) {
    const uint16_t *pl = ain + plane_base(G, T.b, kk);
#pragma unroll
    for (int u = 0; u < kPlaneLoads; ++u) pre[u] = *(const u32x4 *)(pl + src[u]);
  };
  auto store = [&](unsigned char *dst) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kPlaneLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) *(u32x4 *)(dst + (e >> 1) * kCnnCellB + 16 * (e & 1)) = pre[u];
    }
  };
  // plane P into slot(P) (all waves finished reading that slot before the
  // last barrier); the one after it prepared.  Fused: layer 0 of plane P
  // itself runs among the products of the plane before; here the level
  // that layer-0 plane P + 1 adds to the ring (read in the next step) is
  // stored, into the slot of the level two below the ones read in this
  // step, and the level plane P + 2 adds is fetched.
  auto produce = [&](int P) __attribute__((always_inline)) {
    if constexpr (FUSED) {
      if (P + 1 <= T.k1) {
        if (clampz(P + 1) > clampz(P)) store_level(clampz(P + 1) + 1);
        if (P + 2 <= T.k1 && clampz(P + 2) > clampz(P + 1)) fetch_level(clampz(P + 2) + 1);
      }
    } else {
      store(lds[slot(P)]);
      if (P + 1 <= T.k1) fetch(P + 1);
    }
  };
  if constexpr (FUSED) {
    // the levels of layer-0 planes k0 - 1 and k0; the one plane k0 + 1 adds
    const int c0 = clampz(T.k0 - 1);
    for (int u = c0 - 1; u <= clampz(T.k0) + 1; ++u) {
      fetch_level(u);
      store_level(u);
    }
    if (T.k0 + 1 <= T.k1 && clampz(T.k0 + 1) > clampz(T.k0)) fetch_level(clampz(T.k0 + 1) + 1);
    __syncthreads();
    layer0(T.k0 - 1);
  } else {
    fetch(T.k0 - 1);
    store(lds[slot(T.k0 - 1)]);
    fetch(T.k0);
  }
  __syncthreads();

  // Plane p with the accumulators of levels p - 1 (lo), p (mid), p + 1
  // (hi); MODE 1: hi only.  Produces plane p + 1, emits level p - 1 and
  // clears lo (the next plane's hi).  Fused: the layer-0 chains of plane
  // p + 1 are spread over the pairs so that their latency overlaps the
  // products; at p = k1 they fill a slot nobody reads (the stale input set
  // there is a finite earlier one).
  auto plane = [&](auto mode, int p, floatx4(&lo)[4], floatx4(&mid)[4],
                   floatx4(&hi)[4]) __attribute__((always_inline)) {
    constexpr int MODE = decltype(mode)::value;
    const unsigned char *cur = lds[slot(p)];
#pragma unroll
    for (int m = 0; m < kCnnPairs; ++m) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bf16x8 b = *(const bf16x8 *)(cur + poff[m] + c * 16 * kCnnCellB);
        if constexpr (MODE == 0) {
          lo[c] = mfma32(wa[2][m], b, lo[c]);
          mid[c] = mfma32(wa[1][m], b, mid[c]);
        }
        hi[c] = mfma32(wa[0][m], b, hi[c]);
      }
      if constexpr (FUSED) {
        layer0_chain(m, p + 1);
        if (m == 0) layer0_chain(5, p + 1);
        if (m == 1 && wv == 0) layer0_chain(6, p + 1);
      }
    }
    if (p < T.k1) produce(p + 1);
    const int o = p - 1;
    if (o >= T.k0 && oy < G.nyo) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int ox = T.ox0 + 16 * c + row;
        if (ox < G.nxo) {
          const uint32_t l2 = f2bf2(leaky(lo[c][0] + bq[0], alpha),
                                    leaky(lo[c][1] + bq[1], alpha));
          const uint32_t h2 = f2bf2(leaky(lo[c][2] + bq[2], alpha),
                                    leaky(lo[c][3] + bq[3], alpha));
          const int64_t q = (((int64_t)T.b * G.nz + o) * G.nyo + oy) * G.nxo + ox;
          *(uint2 *)(aout + q * kCnnCh + 4 * quad) = make_uint2(l2, h2);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) lo[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    __syncthreads();
  };
  floatx4 a0[4], a1[4], a2[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    a0[c] = floatx4{0.f, 0.f, 0.f, 0.f};
    a1[c] = a0[c];
    a2[c] = a0[c];
  }
  // plane k0 - 1 feeds level k0 only; the later planes run all three
  // products (at planes k0 and k1 one or two of them belong to levels
  // outside the chunk and are dropped), the accumulators rotating roles
  // every plane: three planes per trip
  plane(std::integral_constant<int, 1>{}, T.k0 - 1, a0, a1, a2);
  for (int p = T.k0;; p += 3) {
    plane(std::integral_constant<int, 0>{}, p, a1, a2, a0);
    if (p + 1 > T.k1) break;
    plane(std::integral_constant<int, 0>{}, p + 1, a2, a0, a1);
    if (p + 2 > T.k1) break;
    plane(std::integral_constant<int, 0>{}, p + 2, a0, a1, a2);
    if (p + 3 > T.k1) break;
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
  if (!T.valid) return;  // the whole block
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
        const uint32_t lo = f2bf2(leaky(acc[0] + bq[0], alpha),
                                  leaky(acc[1] + bq[1], alpha));
        const uint32_t hi = f2bf2(leaky(acc[2] + bq[2], alpha),
                                  leaky(acc[3] + bq[3], alpha));
        const int64_t q = (((int64_t)T.b * G.nz + k) * G.nyo + oy) * G.nxo + ox;
        *(uint2 *)(aout + q * kCnnCh + 4 * quad) = make_uint2(lo, hi);
      }
    }
  }
}

// Layer 3 (16 -> 1): y = conv(ain) + b.  The activations are the row operand
// (lane l % 16 = cell, as in the layers before) and the weights the column
// operand, whose columns 0..2 carry the three open output levels: with the
// plane counter q = p - (k0 - 1), column j accumulates the levels u = o -
// (k0 - 1) with u = j (mod 3), so at plane q column j takes the tap row dz
// = q - u.  Level p - 1 (column (q + 2) mod 3) is complete after plane p:
// its lanes hold 4 consecutive cells each; they pass them on and clear the
// column.
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
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][kCnnPlane * kCnnCellB];
  __shared__ __attribute__((aligned(16))) float res[4][kCnnTX];  // a finished level per wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, quad = lane >> 4, side = quad >> 1, half = quad & 1;
  const CnnTile Tl = cnn_tile(G, tiles_x, tiles_y, chunks);
  if (!Tl.valid) return;  // the whole block
  const uint16_t *w3 = wbf + cnn_weight_offset(G.inputs, 3);

  // weights: column j = row < 3 holds W3[9 j + t][8 half .. + 7] (dz = j -
  // 1), t = 2 m + side; the other columns are zero
  bf16x8 wb[kCnnPairs];
  uint32_t poff[kCnnPairs];
#pragma unroll
  for (int m = 0; m < kCnnPairs; ++m) {
    const int t = 2 * m + side;
    wb[m] = row < 3 && t < 9 ? load_w8(w3 + (9 * row + t) * kCnnCh + 8 * half) : bf16x8{};
    poff[m] = pair_offset(wv, row, side, half, m);
  }
  const float b3 = params[cnn_bias_offset(G.inputs, 3)];
  const double sd = GUESS ? *s_over_d : 0.0;
  const int oy = Tl.oy0 + wv;

  // plane kk fetched into registers one plane ahead (the loads past the
  // plane repeat its last cell and are not stored), then stored to a slot
  int32_t src[kPlaneLoads];
  plane_sources(G, Tl, src);
  u32x4 pre[kPlaneLoads];
  auto fetch = [&](int kk) __attribute__((always_inline)) {
    const uint16_t *pl = ain + plane_base(G, Tl.b, kk);
#pragma unroll
    for (int u = 0; u < kPlaneLoads; ++u) pre[u] = *(const u32x4 *)(pl + src[u]);
  };
  auto store = [&](unsigned char *slot) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kPlaneLoads; ++u) {
      const int e = threadIdx.x + 256 * u;
      if (e < kCnnPlane * 2) *(u32x4 *)(slot + (e >> 1) * kCnnCellB + 16 * (e & 1)) = pre[u];
    }
  };
  fetch(Tl.k0 - 1);
  store(lds[0]);
  fetch(Tl.k0);
  __syncthreads();

  // Column j of the accumulators holds level p + 1 - j while plane p is
  // applied: plane p adds its dz = j - 1 taps to column j, then level p - 1
  // (column 2) is emitted and every column moves one to the right (lane l
  // takes lane l - 1 of its 16-lane row, column 0 starts from zero), so
  // each level collects its three planes in order with one weight set.
  floatx4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  auto plane = [&](int p) __attribute__((always_inline)) {
    const unsigned char *cur = lds[(p - Tl.k0 + 1) & 1];
    // the lane's output cell of level p - 1 (finished by this plane); its
    // base value is loaded before the products
    const int o = p - 1, ox = Tl.ox0 + lane;
    const bool emit = o >= Tl.k0 && oy < G.nyo && ox < G.nxo;
    const int64_t q = (((int64_t)Tl.b * G.nz + (emit ? o : 0)) * G.nyo + (emit ? oy : 0)) * G.nxo +
                      (emit ? ox : 0);
    T bval = T(0);
    if (GUESS && emit) bval = base[q];
#pragma unroll
    for (int m = 0; m < kCnnPairs; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bf16x8 a = *(const bf16x8 *)(cur + poff[m] + c * 16 * kCnnCellB);
        acc[c] = mfma32(a, wb[m], acc[c]);
      }
    if (p < Tl.k1) {
      store(lds[(p - Tl.k0) & 1]);
      if (p + 1 < Tl.k1) fetch(p + 2);
    }
    // level p - 1 (column 2) through the wave's LDS row, so that lane l
    // writes cell ox0 + l (LDS operations of one wave complete in order)
    if (row == 2) {
#pragma unroll
      for (int c = 0; c < 4; ++c) *(floatx4 *)&res[wv][16 * c + 4 * quad] = acc[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r)  // DPP row_shr:1, zero into lane 0 of each row
        acc[c][r] = __int_as_float(
            __builtin_amdgcn_update_dpp(0, __float_as_int(acc[c][r]), 0x111, 0xF, 0xF, true));
    __builtin_amdgcn_wave_barrier();
    if (emit) {
      const float out = res[wv][lane] + b3;
      if (GUESS)
        guess[q] = (T)((double)bval + sd * (double)out);
      else
        y[q] = out;
    }
    __syncthreads();
  };
  for (int p = Tl.k0 - 1; p <= Tl.k1; ++p) plane(p);
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

template <typename T, bool BASE>
__global__ __launch_bounds__(kBlock) void residual_kernel(Grid g, double ix2, double iy2,
                                                          double iz2, const T *__restrict__ rhs,
                                                          const T *__restrict__ base,
                                                          float *__restrict__ r,
                                                          double *__restrict__ partials) {
  double acc = 0.0;
  // each block takes a run of x rows (xcd_rows), four at a time so that
  // their loads are in flight together (rows past the run repeat its first
  // row and are not counted); level and y index uniform over the block
  const int64_t rows = (int64_t)g.ny * g.nz;
  constexpr int R = 4;
  const RowRange rr = xcd_rows(rows);
  // (level, y row) of row r0 + u, stepped without divisions
  const RowStep rs(g.ny, 1);
  RowPos p0 = rs.at(rr.r0);
  for (int64_t r0 = rr.r0; r0 < rr.r1; r0 += R) {
    RowPos pu[R];
    pu[0] = p0;
#pragma unroll
    for (int u = 1; u < R; ++u) pu[u] = rs.next(pu[u - 1]);
    p0 = rs.next(pu[R - 1]);
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
      const int ip = i + 1 < g.nx ? i + 1 : 0, im = i > 0 ? i - 1 : g.nx - 1;
      double rv[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const bool in = r0 + u < rr.r1;
        const int64_t row = in ? r0 + u : r0;
        const RowPos q = in ? pu[u] : pu[0];
        const int k = q.k, j = q.j;
        double v = (double)rhs[row * g.nx + i];
        if constexpr (BASE) {
          const T *c0 = base + row * g.nx;
          const T *yp = base + ((int64_t)k * g.ny + pwrap(j + 1, g.ny)) * g.nx;
          const T *ym = base + ((int64_t)k * g.ny + pwrap(j - 1, g.ny)) * g.nx;
          const T *zp = base + ((int64_t)zmirror(k + 1, g.nz) * g.ny + j) * g.nx;
          const T *zm = base + ((int64_t)zmirror(k - 1, g.nz) * g.ny + j) * g.nx;
          const double c = c0[i];
          const double lap = ((double)c0[ip] + (double)c0[im] - 2.0 * c) * ix2 +
                             ((double)yp[i] + (double)ym[i] - 2.0 * c) * iy2 +
                             ((double)zp[i] + (double)zm[i] - 2.0 * c) * iz2;
          v -= lap;
        }
        rv[u] = v;
      }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int64_t row = r0 + u;
        if (row < rr.r1) {
          r[row * g.nx + i] = (float)rv[u];
          acc += rv[u] * rv[u];
        }
      }
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
  const unsigned blocks = cnn_blocks((int64_t)G.batch * tiles_x * tiles_y * chunks);
  if (layer == 0) {
    if (G.inputs == 3)
      conv_in_kernel<3><<<blocks, 256, 0, s>>>(G, ain, params, wbf, alpha, aout, tiles_x, tiles_y,
                                               chunks);
    else
      conv_in_kernel<1><<<blocks, 256, 0, s>>>(G, ain, params, wbf, alpha, aout, tiles_x, tiles_y,
                                               chunks);
  } else if (layer < kCnnLayers - 1) {
    conv_mid_kernel<false><<<blocks, 256, 0, s>>>(
        G, ain, nullptr, nullptr, nullptr, nullptr, params + cnn_bias_offset(G.inputs, layer),
        wbf + cnn_weight_offset(G.inputs, layer), alpha, aout, tiles_x, tiles_y, chunks);
  } else {
    conv_out_kernel<float, false><<<blocks, 256, 0, s>>>(G, ain, params, wbf, yout, nullptr,
                                                         nullptr, nullptr, tiles_x, tiles_y,
                                                         chunks);
  }
}

void launch_cnn_in_mid(const CnnGeom &G, const float *r, const double *scale, const float *params,
                       const uint16_t *wbf, float alpha, uint16_t *aout, hipStream_t s) {
  const int tiles_x = (G.nxo + kCnnTX - 1) / kCnnTX, tiles_y = (G.nyo + kCnnTY - 1) / kCnnTY;
  const int chunks = (G.nz + kCnnKC - 1) / kCnnKC;
  const unsigned blocks = cnn_blocks((int64_t)G.batch * tiles_x * tiles_y * chunks);
  conv_mid_kernel<true><<<blocks, 256, 0, s>>>(
      G, nullptr, r, scale, params + cnn_bias_offset(1, 0), wbf + cnn_weight_offset(1, 0),
      params + cnn_bias_offset(1, 1), wbf + cnn_weight_offset(1, 1), alpha, aout, tiles_x, tiles_y,
      chunks);
}

template <typename T>
void launch_cnn_guess(const CnnGeom &G, const uint16_t *ain, const float *params,
                      const uint16_t *wbf, const T *base, const double *s_over_d, T *guess,
                      hipStream_t s) {
  const int tiles_x = (G.nxo + kCnnTX - 1) / kCnnTX, tiles_y = (G.nyo + kCnnTY - 1) / kCnnTY;
  const int chunks = (G.nz + kCnnKC - 1) / kCnnKC;
  const unsigned blocks = cnn_blocks((int64_t)G.batch * tiles_x * tiles_y * chunks);
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
  const double ix2 = 1.0 / (g.dx * g.dx), iy2 = 1.0 / (g.dy * g.dy), iz2 = 1.0 / (g.dz * g.dz);
  if (base)
    residual_kernel<T, true><<<kReduceBlocks, kBlock, 0, s>>>(g, ix2, iy2, iz2, rhs, base, r,
                                                              partials);
  else
    residual_kernel<T, false><<<kReduceBlocks, kBlock, 0, s>>>(g, ix2, iy2, iz2, rhs, base, r,
                                                               partials);
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
