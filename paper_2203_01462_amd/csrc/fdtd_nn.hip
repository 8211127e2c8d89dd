// fdtd_nn.hip -- kernels of the surrogate network: 3x3 convolutions as
// implicit GEMMs on the BF16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32
// accumulation), their data and weight gradients, and the elementwise,
// pooling, head, loss and optimizer kernels around them.
//
// GEMM tiling: a workgroup (4 wavefronts) owns a 64 x 64 output tile and
// walks the reduction dimension in steps of 16, staging both operand tiles
// in LDS (the im2col gather of the 3x3 window happens while staging); each
// wavefront owns 16 output rows and issues four 16x16x16 MFMAs per step.
// MFMA operand layout (wave64): lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and returns D[4(l/16)+j][l%16], j = 0..3.
#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "fdtd_internal.hpp"
#include "fdtd_nn.h"

using namespace fdtd;

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int BS = 256;
constexpr int TM = 64, TN = 64, TK = 16, PAD = 4;

// IEEE binary32 -> bfloat16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// The BF16 output of a convolution: relu(v) in the forward pass; with a mask
// (the BF16 output of the ReLU that produced this convolution's input, in a
// data-gradient pass) the pre-activation gradient v * (mask > 0), the same
// value as the separate ReLU backward of the FP32 v.
__device__ __forceinline__ uint16_t store_a(float v, const uint16_t *__restrict__ mask, size_t o) {
  return mask ? f2bf(bf2f(mask[o]) > 0.f ? v : 0.f) : f2bf(fmaxf(v, 0.f));
}

// Mask values of one 16-channel block of a tiled kernel's outputs: rows
// `row0 + s` (s < 4, pix0 = the first row's pixel offset) at the lane's
// column, channels co0 + 4 kq + j.
__device__ __forceinline__ void load_mask16(uint16_t (&mk)[4][4], int co0, int cout, int kq, size_t pix0, int w,
                                            size_t cs, const uint16_t *__restrict__ mask) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = co0 + 4 * kq + j;
      mk[s][j] = co < cout ? mask[(size_t)co * cs + pix0 + (size_t)s * w] : (uint16_t)0;
    }
}

// Output of that block: z = v (FP32) and/or a = relu(v) (BF16), or with a
// mask (mk loaded by load_mask16) a = v * (mask > 0) (BF16).  The values are
// formed first and stored back to back (a store between loads and arithmetic
// that reuse its registers would wait for it to complete).
__device__ __forceinline__ void tile_out16(const f4 (&acc)[4], const uint16_t (&mk)[4][4], bool masked, int co0,
                                           int cout, int kq, size_t pix0, int w, size_t cs,
                                           const float *__restrict__ bias, float *__restrict__ z,
                                           uint16_t *__restrict__ a) {
  // the lane's four biases, loaded together ahead of the stores
  float bv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bv[j] = (bias && co0 + 4 * kq + j < cout) ? bias[co0 + 4 * kq + j] : 0.f;
  float v[4][4];
  uint16_t b[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[s][j] = acc[s][j] + bv[j];
      b[s][j] = masked ? f2bf(bf2f(mk[s][j]) > 0.f ? v[s][j] : 0.f) : f2bf(fmaxf(v[s][j], 0.f));
    }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int co = co0 + 4 * kq + j;
    if (co >= cout) continue;
    const size_t o = (size_t)co * cs + pix0;
    if (z) {
#pragma unroll
      for (int s = 0; s < 4; ++s) z[o + (size_t)s * w] = v[s][j];
    }
    if (a) {
#pragma unroll
      for (int s = 0; s < 4; ++s) a[o + (size_t)s * w] = b[s][j];
    }
  }
}

__device__ __forceinline__ double block_sum(double v, double *lds) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / 64; ++k) s += lds[k];
  __syncthreads();
  return s;
}

// One 16-step of the K loop: wavefront `wave` multiplies its 16 rows of As
// with the four 16-column blocks of Bs.
__device__ __forceinline__ void mfma_step(const uint16_t (*As)[TK + PAD], const uint16_t (*Bs)[TN + PAD], int wave,
                                          int lane, f4 acc[4]) {
  s4 a;
#pragma unroll
  for (int j = 0; j < 4; ++j) a[j] = (short)As[16 * wave + (lane & 15)][4 * (lane >> 4) + j];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    s4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = (short)Bs[4 * (lane >> 4) + j][16 * s + (lane & 15)];
    acc[s] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[s], 0, 0, 0);
  }
}

// z[co][n][p] = bias[co] + sum_k w[co][k] xhat[k][n][p], k = (ky, kx, ci),
// xhat = the zero-padded 3x3 window of x[ci][n].  Writes z (FP32) and/or
// a = bf16(max(z, 0)).  grid (ceil(HW/64), ceil(cout/64), n).
__global__ void __launch_bounds__(BS) conv_fwd_kernel(int cin, int cout, int h, int w, const uint16_t *__restrict__ x,
                                                     const uint16_t *__restrict__ wt, const float *__restrict__ bias,
                                                     float *__restrict__ z, uint16_t *__restrict__ a,
                                                     const uint16_t *__restrict__ mask) {
  __shared__ uint16_t As[TM][TK + PAD];
  __shared__ uint16_t Bs[TK][TN + PAD];
  const int n = blockIdx.z, nimg = gridDim.z, HW = h * w, K = cin * 9;
  const int p0 = blockIdx.x * TN, co0 = blockIdx.y * TM;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const size_t cs = (size_t)nimg * HW;  // channel stride
  const uint16_t *xn = x + (size_t)n * HW;
  f4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += TK) {
    {
      const int r = t >> 2, c = (t & 3) * 4, co = co0 + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + c + j;
        As[r][c + j] = (co < cout && k < K) ? wt[(size_t)co * K + k] : (uint16_t)0;
      }
    }
    {
      const int kk = t >> 4, c = (t & 15) * 4, k = k0 + kk;
      const int tap = k / cin, ci = k - tap * cin, ky = tap / 3, kx = tap - ky * 3;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = p0 + c + j;
        uint16_t v = 0;
        if (k < K && p < HW) {
          const int y = p / w, xx = p - y * w, iy = y + ky - 1, ix = xx + kx - 1;
          if (iy >= 0 && iy < h && ix >= 0 && ix < w) v = xn[(size_t)ci * cs + iy * w + ix];
        }
        Bs[kk][c + j] = v;
      }
    }
    __syncthreads();
    mfma_step(As, Bs, wave, lane, acc);
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = co0 + 16 * wave + 4 * (lane >> 4) + j, p = p0 + 16 * s + (lane & 15);
      if (co < cout && p < HW) {
        const float v = acc[s][j] + (bias ? bias[co] : 0.f);
        const size_t o = (size_t)co * cs + (size_t)n * HW + p;
        if (z) z[o] = v;
        if (a) a[o] = store_a(v, mask, o);
      }
    }
}

// The same convolution, LDS-tiled for cin % 32 == 0 and h, w multiples of 16,
// on v_mfma_f32_16x16x32_bf16, reading a channel-last copy of the input
// (x[n][y][x][cin], to_nhwc_kernel).  A workgroup owns 16*MT output channels
// x a 16 x 16 pixel tile of one image; per chunk of 32 input channels it
// stages the 18 x 18 halo tile in LDS (a pixel's 32 channels are four
// 16-byte loads; eight channels of one pixel are one 16-byte LDS read) and
// the weights of all nine taps, then each
// wavefront (four pixel rows) runs nine taps x MT x 4 matrix instructions.
// grid ((h/16) * (w/16), ceil(cout / (16*MT)), n).
// Pipelined variant: a workgroup walks `tpw` pixel tiles; the next (tile,
// chunk)'s input (and, with several chunks, its weights) is loaded into
// registers before the current chunk's matrix instructions and written to
// LDS after them; grid (ceil(tiles / tpw), ceil(cout / (16*MT)), n).
constexpr int CC = 32;                  // input channels per chunk
constexpr int XST = 40;                 // LDS stride between staged pixels (80 B: conflict-free 16 B reads)
constexpr int WST = 40;                 // LDS stride between staged (tap, co) weight rows
constexpr int TT = 16, HT = TT + 2;     // output tile side, halo tile side

template <int MT>
__global__ void __launch_bounds__(BS) conv_fwd_mfma_kernel(int cin, int cout, int h, int w,
                                                          const uint16_t *__restrict__ x,
                                                          const uint16_t *__restrict__ wt,
                                                          const float *__restrict__ bias, float *__restrict__ z,
                                                          uint16_t *__restrict__ a,
                                                          const uint16_t *__restrict__ mask) {
  __shared__ __attribute__((aligned(16))) uint16_t Xs[HT * HT * XST];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[9 * 16 * MT * WST];
  const int n = blockIdx.z, nimg = gridDim.z, HW = h * w;
  const int tilesx = w / TT;
  const int y0 = (blockIdx.x / tilesx) * TT, x0 = (blockIdx.x % tilesx) * TT;
  const int co0 = blockIdx.y * 16 * MT;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, l16 = lane & 15, kq = lane >> 4;
  const size_t cs = (size_t)nimg * HW;
  f4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[m][s] = f4{0.f, 0.f, 0.f, 0.f};
  // a data-gradient pass's mask values, loaded first so that they arrive
  // while the tile is staged and multiplied
  const size_t pix0 = (size_t)n * HW + (size_t)(y0 + 4 * wave) * w + x0 + l16;
  const bool masked = a && mask;
  uint16_t mk[MT][4][4];
  if (masked) {
#pragma unroll
    for (int m = 0; m < MT; ++m) load_mask16(mk[m], co0 + 16 * m, cout, kq, pix0, w, cs, mask);
  }
  for (int c0 = 0; c0 < cin; c0 += CC) {
    for (int v = t; v < 9 * 16 * MT * 4; v += BS) {
      const int part = v & 3, row = v >> 2;
      const int tap = row / (16 * MT), col = row - tap * (16 * MT), co = co0 + col;
      uint4 val = {0u, 0u, 0u, 0u};
      if (co < cout) val = *(const uint4 *)(wt + ((size_t)co * 9 + tap) * cin + c0 + 8 * part);
      *(uint4 *)(Ws + row * WST + 8 * part) = val;
    }
    // one halo pixel per thread: its 32 channels, packed into 16-byte LDS writes
    for (int pos = t; pos < HT * HT; pos += BS) {
      const int r = pos / HT, q = pos - r * HT;
      const int iy = y0 - 1 + r, ix = x0 - 1 + q;
      const bool ok = iy >= 0 && iy < h && ix >= 0 && ix < w;
      // channel-last input: the pixel's 32 channels are 64 contiguous bytes
      const uint4 *src = (const uint4 *)(x + ((size_t)n * HW + (ok ? iy * w + ix : 0)) * cin + c0);
#pragma unroll
      for (int c8 = 0; c8 < CC / 8; ++c8)
        *(uint4 *)(Xs + pos * XST + 8 * c8) = ok ? src[c8] : uint4{0u, 0u, 0u, 0u};
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap - 3 * ky;
      bf8 av[MT], bv[4];
#pragma unroll
      for (int m = 0; m < MT; ++m) av[m] = *(const bf8 *)(Ws + (tap * 16 * MT + 16 * m + l16) * WST + 8 * kq);
#pragma unroll
      for (int s = 0; s < 4; ++s) bv[s] = *(const bf8 *)(Xs + ((4 * wave + s + ky) * HT + l16 + kx) * XST + 8 * kq);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[m][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[s], acc[m][s], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < MT; ++m) tile_out16(acc[m], mk[m], masked, co0 + 16 * m, cout, kq, pix0, w, cs, bias, z, a);
}

// The same with the staging software-pipelined (see above): faster on the
// deep layers with a few pixel tiles and several channel chunks, slower on
// the wide ones (its prefetch registers leave one wavefront per SIMD).
template <int MT>
__global__ void __launch_bounds__(BS) conv_fwd_mfma_pipe_kernel(int cin, int cout, int h, int w,
                                                               const uint16_t *__restrict__ x,
                                                               const uint16_t *__restrict__ wt,
                                                               const float *__restrict__ bias,
                                                               float *__restrict__ z, uint16_t *__restrict__ a,
                                                               const uint16_t *__restrict__ mask, const int tpw) {
  __shared__ __attribute__((aligned(16))) uint16_t Xs[HT * HT * XST];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[9 * 16 * MT * WST];
  constexpr int NXP = (HT * HT + BS - 1) / BS;           // halo pixels per thread (2)
  constexpr int NWV = (9 * 16 * MT * 4 + BS - 1) / BS;   // 16-byte weight vectors per thread
  const int n = blockIdx.z, nimg = gridDim.z, HW = h * w;
  const int tilesx = w / TT, tiles = (h / TT) * tilesx;
  const int tb = blockIdx.x * tpw, te = min(tiles, tb + tpw);
  const int nch = cin / CC, steps = (te - tb) * nch;  // (pixel tile, channel chunk), chunk fastest
  const int co0 = blockIdx.y * 16 * MT;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, l16 = lane & 15, kq = lane >> 4;
  const size_t cs = (size_t)nimg * HW;
  uint32_t xr[NXP][CC / 2];
  uint4 wr[NWV];
  // global -> registers for step (tile, c0); registers -> LDS after the barrier
  auto load_x = [&](int tile, int c0) {
    const int y0 = (tile / tilesx) * TT, x0 = (tile % tilesx) * TT;
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      const int pos = t + k * BS;
      const int r = pos / HT, q = pos - r * HT;
      const int iy = y0 - 1 + r, ix = x0 - 1 + q;
      const bool ok = pos < HT * HT && iy >= 0 && iy < h && ix >= 0 && ix < w;
      const uint4 *src = (const uint4 *)(x + ((size_t)n * HW + (ok ? iy * w + ix : 0)) * cin + c0);
#pragma unroll
      for (int c8 = 0; c8 < CC / 8; ++c8) {
        const uint4 v = ok ? src[c8] : uint4{0u, 0u, 0u, 0u};
        xr[k][4 * c8] = v.x;
        xr[k][4 * c8 + 1] = v.y;
        xr[k][4 * c8 + 2] = v.z;
        xr[k][4 * c8 + 3] = v.w;
      }
    }
  };
  auto store_x = [&]() {
#pragma unroll
    for (int k = 0; k < NXP; ++k) {
      const int pos = t + k * BS;
      if (pos < HT * HT) {
#pragma unroll
        for (int c8 = 0; c8 < CC / 8; ++c8)
          *(uint4 *)(Xs + pos * XST + 8 * c8) = uint4{xr[k][4 * c8], xr[k][4 * c8 + 1], xr[k][4 * c8 + 2], xr[k][4 * c8 + 3]};
      }
    }
  };
  auto load_w = [&](int c0) {
#pragma unroll
    for (int k = 0; k < NWV; ++k) {
      const int v = t + k * BS;
      const int part = v & 3, row = v >> 2;
      const int tap = row / (16 * MT), col = row - tap * (16 * MT), co = co0 + col;
      wr[k] = uint4{0u, 0u, 0u, 0u};
      if (v < 9 * 16 * MT * 4 && co < cout) wr[k] = *(const uint4 *)(wt + ((size_t)co * 9 + tap) * cin + c0 + 8 * part);
    }
  };
  auto store_w = [&]() {
#pragma unroll
    for (int k = 0; k < NWV; ++k) {
      const int v = t + k * BS;
      if (v < 9 * 16 * MT * 4) *(uint4 *)(Ws + (v >> 2) * WST + 8 * (v & 3)) = wr[k];
    }
  };
  if (steps <= 0) return;
  f4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[m][s] = f4{0.f, 0.f, 0.f, 0.f};
  load_w(0);
  load_x(tb, 0);
  for (int st = 0; st < steps; ++st) {
    const int tile = tb + st / nch, ch = st - (st / nch) * nch;
    if (st == 0 || nch > 1) store_w();  // one chunk: the weights stay for every tile
    store_x();
    __syncthreads();
    if (st + 1 < steps) {  // the next step's loads fly while the matrix cores work
      const int nt = tb + (st + 1) / nch, nc = (st + 1) - ((st + 1) / nch) * nch;
      if (nch > 1) load_w(nc * CC);
      load_x(nt, nc * CC);
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap - 3 * ky;
      bf8 av[MT], bv[4];
#pragma unroll
      for (int m = 0; m < MT; ++m) av[m] = *(const bf8 *)(Ws + (tap * 16 * MT + 16 * m + l16) * WST + 8 * kq);
#pragma unroll
      for (int s = 0; s < 4; ++s) bv[s] = *(const bf8 *)(Xs + ((4 * wave + s + ky) * HT + l16 + kx) * XST + 8 * kq);
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[m][s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[m], bv[s], acc[m][s], 0, 0, 0);
    }
    if (ch == nch - 1) {  // the tile's last chunk: write it out
      const int y0 = (tile / tilesx) * TT, x0 = (tile % tilesx) * TT;
      const size_t pix0 = (size_t)n * HW + (size_t)(y0 + 4 * wave) * w + x0 + l16;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        uint16_t mk[4][4];
        if (a && mask) load_mask16(mk, co0 + 16 * m, cout, kq, pix0, w, cs, mask);
        tile_out16(acc[m], mk, a && mask, co0 + 16 * m, cout, kq, pix0, w, cs, bias, z, a);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[m][s] = f4{0.f, 0.f, 0.f, 0.f};
      }
    }
    __syncthreads();
  }
}

// Channel-last copy of a [c][n][hw] BF16 tensor: y[(img hw + p) c + ch].
// grid (hw / 64, c / 32, n): a workgroup moves 64 pixels x 32 channels
// through LDS, reading rows of pixels and writing 64-byte channel runs.
__global__ void __launch_bounds__(BS) to_nhwc_kernel(int c, int hw, const uint16_t *__restrict__ x,
                                                     uint16_t *__restrict__ y) {
  __shared__ uint16_t tile[32][64 + 2];
  const int p0 = blockIdx.x * 64, c0 = blockIdx.y * 32, img = blockIdx.z, nimg = gridDim.z;
  const int t = threadIdx.x;
  const size_t cs = (size_t)nimg * hw;
  {
    const int p = t & 63, g = t >> 6;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int ch = g * 8 + k;
      tile[ch][p] = x[(size_t)(c0 + ch) * cs + (size_t)img * hw + p0 + p];
    }
  }
  __syncthreads();
  const int p = t >> 2, part = t & 3;
  uint32_t pk[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    pk[j] = (uint32_t)tile[part * 8 + 2 * j][p] | ((uint32_t)tile[part * 8 + 2 * j + 1][p] << 16);
  *(uint4 *)(y + ((size_t)img * hw + p0 + p) * c + c0 + part * 8) = uint4{pk[0], pk[1], pk[2], pk[3]};
}

// The convolution of a one-channel input (cout <= 64): a workgroup of 64 x 4
// pixels stages its 66 x 6 input halo and the weights in LDS; each thread
// forms its pixel's cout outputs as FP32 sums over the taps in order (plus
// the bias), written as z and/or a (store_a).  grid (ceil(w/64), ceil(h/4), n).
__global__ void __launch_bounds__(BS) conv1_fwd_kernel(int cout, int h, int w, const uint16_t *__restrict__ x,
                                                      const uint16_t *__restrict__ wt, const float *__restrict__ bias,
                                                      float *__restrict__ z, uint16_t *__restrict__ a,
                                                      const uint16_t *__restrict__ mask) {
  __shared__ float xs[6][66];
  __shared__ float ws[64 * 9];
  const int n = blockIdx.z, nimg = gridDim.z, HW = h * w;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 4;
  const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
  for (int i = t; i < 6 * 66; i += BS) {
    const int r = i / 66, q = i - r * 66, iy = y0 - 1 + r, ix = x0 - 1 + q;
    xs[r][q] = (iy >= 0 && iy < h && ix >= 0 && ix < w) ? bf2f(x[(size_t)n * HW + (size_t)iy * w + ix]) : 0.f;
  }
  for (int i = t; i < cout * 9; i += BS) ws[i] = bf2f(wt[i]);
  __syncthreads();
  const int xx = x0 + lx, yy = y0 + ly;
  if (xx >= w || yy >= h) return;
  float xn[9];
#pragma unroll
  for (int tp = 0; tp < 9; ++tp) xn[tp] = xs[ly + tp / 3][lx + tp % 3];
  const size_t cs = (size_t)nimg * HW, pix = (size_t)n * HW + (size_t)yy * w + xx;
  for (int co = 0; co < cout; ++co) {
    float v = 0.f;
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) v = fmaf(ws[co * 9 + tp], xn[tp], v);
    v += bias ? bias[co] : 0.f;
    const size_t o = (size_t)co * cs + pix;
    if (z) z[o] = v;
    if (a) a[o] = store_a(v, mask, o);
  }
}

// Device buffer for the channel-last copy of a convolution input, one per
// (device, stream) so that convolutions on different streams never share it;
// kept until the process ends, grown (after the device has drained the work
// that may still read it) to the largest request.
uint16_t *nhwc_buffer(size_t elems, hipStream_t s) {
  int dev = 0;
  FDTD_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> bufs;
  std::lock_guard<std::mutex> lock(mu);
  auto &b = bufs[{dev, s}];
  if (b.second < elems) {
    if (b.first) {
      FDTD_HIP(hipDeviceSynchronize());
      FDTD_HIP(hipFree(b.first));
    }
    b.first = nullptr;
    b.second = 0;
    FDTD_HIP(hipMalloc(&b.first, elems * sizeof(uint16_t)));
    b.second = elems;
  }
  return static_cast<uint16_t *>(b.first);
}

// One forward convolution launch: the LDS-tiled kernel where the shape and
// the weight alignment allow it (its input staged from a channel-last copy,
// 16-byte loads of a pixel's channels), else the generic one.
void launch_conv(int n, int cin, int cout, int h, int w, const uint16_t *x, const uint16_t *wt, const float *bias,
                 float *z, uint16_t *a, const uint16_t *mask, hipStream_t s) {
  if (cin == 1 && cout <= 64) {
    hipLaunchKernelGGL(conv1_fwd_kernel, dim3((w + 63) / 64, (h + 3) / 4, n), dim3(BS), 0, s, cout, h, w, x, wt, bias,
                       z, a, mask);
    return;
  }
  if (cin % CC == 0 && h % TT == 0 && w % TT == 0 && ((uintptr_t)wt & 15) == 0) {
    const int tiles = (h / TT) * (w / TT), cot = cout <= 32 ? (cout + 31) / 32 : (cout + 63) / 64;
    uint16_t *xh = nhwc_buffer((size_t)n * cin * h * w, s);
    hipLaunchKernelGGL(to_nhwc_kernel, dim3(h * w / 64, cin / 32, n), dim3(BS), 0, s, cin, h * w, x, xh);
    if (tiles <= 4 && cin > CC) {  // deep layers: pipelined staging, one tile per workgroup (measured)
      const dim3 g(tiles, cot, n);
      if (cout <= 32)
        hipLaunchKernelGGL((conv_fwd_mfma_pipe_kernel<2>), g, dim3(BS), 0, s, cin, cout, h, w, xh, wt, bias, z,
                           a, mask, 1);
      else
        hipLaunchKernelGGL((conv_fwd_mfma_pipe_kernel<4>), g, dim3(BS), 0, s, cin, cout, h, w, xh, wt, bias, z,
                           a, mask, 1);
      return;
    }
    const dim3 g(tiles, cot, n);
    if (cout <= 32)
      hipLaunchKernelGGL((conv_fwd_mfma_kernel<2>), g, dim3(BS), 0, s, cin, cout, h, w, xh, wt, bias, z, a, mask);
    else
      hipLaunchKernelGGL((conv_fwd_mfma_kernel<4>), g, dim3(BS), 0, s, cin, cout, h, w, xh, wt, bias, z, a, mask);
    return;
  }
  const dim3 g((h * w + TN - 1) / TN, (cout + TM - 1) / TM, n);
  hipLaunchKernelGGL(conv_fwd_kernel, g, dim3(BS), 0, s, cin, cout, h, w, x, wt, bias, z, a, mask);
}

// Partial weight gradients over one range of pixels q = (n, p) of the batch:
// part[split][co][k] = sum_q dz[co][q] xhat[k][q].  grid (ceil(K/64), ceil(cout/64), splits).
__global__ void __launch_bounds__(BS) conv_wgrad_kernel(int nimg, int cin, int cout, int h, int w,
                                                       const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz,
                                                       float *__restrict__ part, int chunk) {
  __shared__ uint16_t As[TM][TK + PAD];  // dz: co x q
  __shared__ uint16_t Bs[TK][TN + PAD];  // xhat: q x k
  const int HW = h * w, K = cin * 9;
  const int64_t P = (int64_t)nimg * HW;
  const int k0 = blockIdx.x * TN, co0 = blockIdx.y * TM, split = blockIdx.z;
  const int64_t qb = (int64_t)split * chunk, qe = min(P, qb + chunk);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  f4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = f4{0.f, 0.f, 0.f, 0.f};
  for (int64_t q0 = qb; q0 < qe; q0 += TK) {
    {
      const int r = t >> 2, c = (t & 3) * 4, co = co0 + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t q = q0 + c + j;
        As[r][c + j] = (co < cout && q < qe) ? dz[(size_t)co * P + q] : (uint16_t)0;
      }
    }
    {
      const int qq = t >> 4, c = (t & 15) * 4;
      const int64_t q = q0 + qq;
      const bool qok = q < qe;
      const int64_t n = qok ? q / HW : 0;
      const int p = qok ? (int)(q - n * HW) : 0;
      const int y = p / w, xx = p - y * w;
      const uint16_t *xn = x + (size_t)n * HW;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + c + j;
        uint16_t v = 0;
        if (qok && k < K) {
          const int tap = k / cin, ci = k - tap * cin, ky = tap / 3, kx = tap - ky * 3;
          const int iy = y + ky - 1, ix = xx + kx - 1;
          if (iy >= 0 && iy < h && ix >= 0 && ix < w) v = xn[(size_t)ci * P + iy * w + ix];
        }
        Bs[qq][c + j] = v;
      }
    }
    __syncthreads();
    mfma_step(As, Bs, wave, lane, acc);
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int co = co0 + 16 * wave + 4 * (lane >> 4) + j, k = k0 + 16 * s + (lane & 15);
      if (co < cout && k < K) part[((size_t)split * cout + co) * K + k] = acc[s][j];
    }
}

// Weight gradient, LDS-tiled for cin % 32 == 0, h % 8 == 0, w % 16 == 0 and
// 16-byte aligned x and dz:
// part[split][co][tap][ci] = sum over the split's pixel tiles of
// dz[co][q] x[ci][q shifted by tap] (rows `stride` floats apart).  A
// workgroup owns CT (64 or 32) output channels x 32 input channels x 9 taps
// and walks 8 x 16 pixel tiles; the reduction runs over pixels (32 per
// matrix instruction), so both operands are staged pixel-contiguous: dz rows
// as they are, and the input tile three times, shifted by kx = 0, 1, 2, so
// every 16-byte fragment read stays aligned.  CT = 64: wavefront w owns
// output channels 16w..16w+15 and both 16-channel halves of the input chunk
// (2 x 9 accumulator tiles); CT = 32 (layers with at most 32 output
// channels): output channels 16(w & 1).. and input half w >> 1 (1 x 9).
// With bpart, the workgroups of the first input chunk also write the
// split's bias partial sums bpart[split * stride + co] = sum of dz[co][q]
// over its tiles.  grid (ceil(cout/CT), cin/32, splits).
constexpr int GY = 8, GX = 16, GP = GY * GX;  // pixel tile
constexpr int DST = GP + 8;                   // LDS stride of staged dz rows
constexpr int XCI = (GY + 2) * GX + 8;        // LDS stride per input channel of a shifted copy

template <int CT>
__global__ void __launch_bounds__(BS) conv_wgrad_mfma_kernel(int nimg, int cin, int cout, int h, int w,
                                                            const uint16_t *__restrict__ x,
                                                            const uint16_t *__restrict__ dz,
                                                            float *__restrict__ part, int64_t stride,
                                                            int tiles_per_split, float *__restrict__ bpart) {
  constexpr int NT = CT / 32;           // 16-channel input halves per wavefront
  constexpr int DV = CT * GY * 2 / BS;  // 16-byte dz vectors per thread and tile
  __shared__ __attribute__((aligned(16))) uint16_t Ds[CT * DST];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[3 * 32 * XCI];
  const int HW = h * w;
  const size_t P = (size_t)nimg * HW;
  const int co0 = blockIdx.x * CT, ci0 = blockIdx.y * 32, split = blockIdx.z;
  const int tx_n = w / GX, tiles_img = (h / GY) * tx_n, tiles = nimg * tiles_img;
  const int T0 = split * tiles_per_split, T1 = min(tiles, T0 + tiles_per_split);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, l16 = lane & 15, kq = lane >> 4;
  const int cw = CT == 64 ? wave : (wave & 1), nb = CT == 64 ? 0 : (wave >> 1);
  const bool with_bias = bpart != nullptr && blockIdx.y == 0;
  f4 acc[NT][9];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) acc[nt][tp] = f4{0.f, 0.f, 0.f, 0.f};
  float bacc[DV];
#pragma unroll
  for (int k = 0; k < DV; ++k) bacc[k] = 0.f;
  // A tile's global loads, issued together into registers: the dz rows (CT
  // channels x 8 rows x 16 pixels as 16-byte vectors) and the input halo
  // rows y0-1 .. y0+8 of the 32 channels (one row per thread and pass: the
  // 16 interior pixels as two 16-byte vectors plus the two halo pixels).
  // The next tile's loads fly while the current tile's matrix instructions run.
  constexpr int XR = (32 * (GY + 2) + BS - 1) / BS;
  uint4 dv[DV], xa[XR], xb[XR];
  uint32_t xl[XR], xr[XR];
  auto load_tile = [&](int T) {
    const int n = T / tiles_img, rem = T - n * tiles_img;
    const int y0 = (rem / tx_n) * GY, x0 = (rem % tx_n) * GX;
#pragma unroll
    for (int k = 0; k < DV; ++k) {
      const int v = t + k * BS;
      const int half = v & 1, r = (v >> 1) & (GY - 1), co = co0 + (v >> 4);
      dv[k] = uint4{0u, 0u, 0u, 0u};
      if (co < cout) dv[k] = *(const uint4 *)(dz + (size_t)co * P + (size_t)n * HW + (size_t)(y0 + r) * w + x0 + 8 * half);
    }
#pragma unroll
    for (int q = 0; q < XR; ++q) {
      const int rr = t + q * BS;
      xa[q] = xb[q] = uint4{0u, 0u, 0u, 0u};
      xl[q] = xr[q] = 0u;
      const int c = rr / (GY + 2), r = rr - c * (GY + 2), iy = y0 - 1 + r;
      if (rr < 32 * (GY + 2) && iy >= 0 && iy < h) {
        const uint16_t *row = x + (size_t)(ci0 + c) * P + (size_t)n * HW + (size_t)iy * w;
        xa[q] = *(const uint4 *)(row + x0);
        xb[q] = *(const uint4 *)(row + x0 + 8);
        if (x0 > 0) xl[q] = row[x0 - 1];
        if (x0 + GX < w) xr[q] = row[x0 + GX];
      }
    }
  };
  // ... and their LDS copies: dz rows as they are, the input rows three
  // times, shifted by kx (copy kx, pixel q = input column x0 - 1 + q + kx)
  auto store_tile = [&]() {
#pragma unroll
    for (int k = 0; k < DV; ++k) {
      const int v = t + k * BS;
      const int half = v & 1, r = (v >> 1) & (GY - 1), c = v >> 4;
      *(uint4 *)(Ds + c * DST + r * GX + 8 * half) = dv[k];
      if (with_bias) {
        const uint32_t u[4] = {dv[k].x, dv[k].y, dv[k].z, dv[k].w};
        float s8 = 0.f;
#pragma unroll
        for (int j = 0; j < 4; ++j) s8 += bf2f((uint16_t)(u[j] & 0xffffu)) + bf2f((uint16_t)(u[j] >> 16));
        bacc[k] += s8;
      }
    }
#pragma unroll
    for (int q = 0; q < XR; ++q) {
      const int rr = t + q * BS;
      if (rr >= 32 * (GY + 2)) continue;
      const int c = rr / (GY + 2), r = rr - c * (GY + 2);
      const uint32_t W[8] = {xa[q].x, xa[q].y, xa[q].z, xa[q].w, xb[q].x, xb[q].y, xb[q].z, xb[q].w};
      uint32_t S0[8], S2[8];
      S0[0] = xl[q] | (W[0] << 16);
#pragma unroll
      for (int k = 1; k < 8; ++k) S0[k] = (W[k - 1] >> 16) | (W[k] << 16);
#pragma unroll
      for (int k = 0; k < 7; ++k) S2[k] = (W[k] >> 16) | (W[k + 1] << 16);
      S2[7] = (W[7] >> 16) | (xr[q] << 16);
      uint16_t *d0 = Xs + (0 * 32 + c) * XCI + r * GX;
      uint16_t *d1 = Xs + (1 * 32 + c) * XCI + r * GX;
      uint16_t *d2 = Xs + (2 * 32 + c) * XCI + r * GX;
      *(uint4 *)d0 = uint4{S0[0], S0[1], S0[2], S0[3]};
      *(uint4 *)(d0 + 8) = uint4{S0[4], S0[5], S0[6], S0[7]};
      *(uint4 *)d1 = uint4{W[0], W[1], W[2], W[3]};
      *(uint4 *)(d1 + 8) = uint4{W[4], W[5], W[6], W[7]};
      *(uint4 *)d2 = uint4{S2[0], S2[1], S2[2], S2[3]};
      *(uint4 *)(d2 + 8) = uint4{S2[4], S2[5], S2[6], S2[7]};
    }
  };
  if (T0 < T1) load_tile(T0);
  for (int T = T0; T < T1; ++T) {
    store_tile();
    __syncthreads();
    if (T + 1 < T1) load_tile(T + 1);
#pragma unroll
    for (int ks = 0; ks < GP / 32; ++ks) {
      const int py = 2 * ks + (kq >> 1), px = 8 * (kq & 1);
      const bf8 av = *(const bf8 *)(Ds + (16 * cw + l16) * DST + 32 * ks + 8 * kq);
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) {
        const int ky = tp / 3, kx = tp - 3 * ky;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const bf8 bv = *(const bf8 *)(Xs + (kx * 32 + 16 * (nb + nt) + l16) * XCI + (py + ky) * GX + px);
          acc[nt][tp] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt][tp], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = co0 + 16 * cw + 4 * kq + j, ci = ci0 + 16 * (nb + nt) + l16;
        if (co < cout) part[(size_t)split * stride + ((size_t)co * 9 + tp) * cin + ci] = acc[nt][tp][j];
      }
  if (with_bias) {
    // the 16 consecutive lanes that staged one channel's rows, summed in a
    // fixed butterfly order
#pragma unroll
    for (int k = 0; k < DV; ++k) {
      float v = bacc[k];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 16);
      const int co = co0 + (t >> 4) + 16 * k;
      if ((t & 15) == 0 && co < cout) bpart[(size_t)split * stride + co] = v;
    }
  }
}

// Weight gradient of a layer with one input channel and at most 32 output
// channels (the network's first layer), h % 8 == 0, w % 64 == 0:
// part[split * stride + co * 9 + tap] = sum over the split's 8 x 64 pixel
// tiles of dz[co][q] x[q shifted by tap], bpart[split * stride + co] = the
// sum of dz[co][q] (FP32).  Wavefront wv owns channels 8 wv .. 8 wv + 7, its
// lanes the tile's columns; a fixed butterfly combines the lanes' sums.
// grid (splits).
constexpr int C1Y = 8;
__global__ void __launch_bounds__(BS) conv1_wgrad_kernel(int nimg, int cout, int h, int w,
                                                        const uint16_t *__restrict__ x, const uint16_t *__restrict__ dz,
                                                        float *__restrict__ part, int64_t stride, int tiles_per_split,
                                                        float *__restrict__ bpart) {
  __shared__ float xs[C1Y + 2][66];
  const int HW = h * w;
  const size_t P = (size_t)nimg * HW;
  const int tx = w / 64, tiles_img = (h / C1Y) * tx, tiles = nimg * tiles_img;
  const int split = blockIdx.x, T0 = split * tiles_per_split, T1 = min(tiles, T0 + tiles_per_split);
  const int t = threadIdx.x, wv = t >> 6, lane = t & 63;
  float acc[8][9], bacc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    bacc[c] = 0.f;
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) acc[c][tp] = 0.f;
  }
  for (int T = T0; T < T1; ++T) {
    const int n = T / tiles_img, rem = T - n * tiles_img;
    const int y0 = (rem / tx) * C1Y, x0 = (rem % tx) * 64;
    __syncthreads();  // the previous tile's rows are read
    for (int i = t; i < (C1Y + 2) * 66; i += BS) {
      const int r = i / 66, q = i - r * 66, iy = y0 - 1 + r, ix = x0 - 1 + q;
      xs[r][q] = (iy >= 0 && iy < h && ix >= 0 && ix < w) ? bf2f(x[(size_t)n * HW + (size_t)iy * w + ix]) : 0.f;
    }
    __syncthreads();
#pragma unroll 2
    for (int r = 0; r < C1Y; ++r) {
      float xn[9];
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) xn[tp] = xs[r + tp / 3][lane + tp % 3];
      const size_t pix = (size_t)n * HW + (size_t)(y0 + r) * w + x0 + lane;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int co = 8 * wv + c;
        const float d = co < cout ? bf2f(dz[(size_t)co * P + pix]) : 0.f;
        bacc[c] += d;
#pragma unroll
        for (int tp = 0; tp < 9; ++tp) acc[c][tp] = fmaf(d, xn[tp], acc[c][tp]);
      }
    }
  }
  // reduce all 80 sums first, then store them back to back
#pragma unroll
  for (int c = 0; c < 8; ++c) {
#pragma unroll
    for (int tp = 0; tp < 9; ++tp)
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc[c][tp] += __shfl_xor(acc[c][tp], o, 64);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bacc[c] += __shfl_xor(bacc[c], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int co = 8 * wv + c;
      if (co >= cout) continue;
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) part[(size_t)split * stride + co * 9 + tp] = acc[c][tp];
      if (bpart) bpart[(size_t)split * stride + co] = bacc[c];
    }
  }
}

// Split plan of the weight gradient: which kernel, how many partial sums,
// pixels (generic) or pixel tiles (tiled) per split.
struct WgradPlan {
  bool tiled, c1;  // LDS-tiled matrix-core kernel; one-input-channel kernel
  int splits, chunk;
};

// Output-channel tile of the tiled weight gradient.
inline int wgrad_ct(int cout) { return cout <= 32 ? 32 : 64; }

// About 768 workgroups in flight (three per CU), at least two pixel tiles
// per tiled workgroup so the partial sums stay few.
WgradPlan wgrad_plan(int n, int cin, int cout, int h, int w) {
  WgradPlan pl{};
  if (cin == 1 && cout <= 32 && h % C1Y == 0 && w % 64 == 0) {
    const int tiles = n * (h / C1Y) * (w / 64);
    pl.c1 = true;
    pl.chunk = std::min(2, tiles);
    pl.splits = (tiles + pl.chunk - 1) / pl.chunk;
    return pl;
  }
  if (cin % 32 == 0 && h % GY == 0 && w % GX == 0) {
    const int ct = wgrad_ct(cout);
    const int groups = ((cout + ct - 1) / ct) * (cin / 32);
    const int tiles = n * (h / GY) * (w / GX);
    const int want = std::max(1, (768 + groups - 1) / groups);
    const int per = std::max(std::min(2, tiles), (tiles + want - 1) / want);
    pl.tiled = true;
    pl.chunk = per;
    pl.splits = (tiles + per - 1) / per;
    return pl;
  }
  const int64_t P = (int64_t)n * h * w;
  const int64_t groups = (int64_t)((cin * 9 + TN - 1) / TN) * ((cout + TM - 1) / TM);
  const int64_t want = std::max<int64_t>(1, (768 + groups - 1) / groups);
  pl.tiled = false;
  pl.splits = (int)std::min<int64_t>(want, std::max<int64_t>(1, (P + 255) / 256));
  int64_t chunk = (P + pl.splits - 1) / pl.splits;
  chunk = (chunk + TK - 1) / TK * TK;
  pl.chunk = (int)chunk;
  pl.splits = (int)((P + chunk - 1) / chunk);
  return pl;
}

// Pixel ranges of the bias-gradient reduction of the generic kernel.
int64_t bias_ranges(int64_t P) { return std::min<int64_t>(64, std::max<int64_t>(1, (P + 16383) / 16384)); }

// out[i] = sum over k < splits of part[k * stride + i], i < m.  G groups of
// consecutive splits per output, each summed in split order (the unrolled
// loads are issued ahead; the additions keep their order), then the G group
// sums in group order: a fixed order for a given split count, with G
// wavefronts' loads in flight per output row when the splits are many.
// grid ceil(m / 64), 64 G threads.
template <int G>
__global__ void __launch_bounds__(64 * G) split_sum_kernel(const float *__restrict__ part, int splits, int64_t stride,
                                                          int64_t m, float *__restrict__ out) {
  __shared__ float red[G][64];
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + o;
  const int k0 = (int)((int64_t)splits * g / G), k1 = (int)((int64_t)splits * (g + 1) / G);
  float s = 0.f;
  if (i < m) {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) s += part[(size_t)k * stride + i];
  }
  if constexpr (G == 1) {
    if (i < m) out[i] = s;
  } else {
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && i < m) {
      float r = red[0][o];
#pragma unroll
      for (int q = 1; q < G; ++q) r += red[q][o];
      out[i] = r;
    }
  }
}

void launch_split_sum(const float *part, int splits, int64_t stride, int64_t m, float *out, hipStream_t s) {
  const dim3 g((unsigned)((m + 63) / 64));
  if (splits >= 64)
    hipLaunchKernelGGL(split_sum_kernel<16>, g, dim3(64 * 16), 0, s, part, splits, stride, m, out);
  else if (splits >= 16)
    hipLaunchKernelGGL(split_sum_kernel<4>, g, dim3(64 * 4), 0, s, part, splits, stride, m, out);
  else
    hipLaunchKernelGGL(split_sum_kernel<1>, g, dim3(64), 0, s, part, splits, stride, m, out);
}

// Partial bias gradients: part[b][co] = sum of dz[co][q] over pixel range b
// (FP64 within the range).  grid (cout, ranges).
__global__ void __launch_bounds__(BS) bias_grad_kernel(int64_t P, int64_t chunk, const uint16_t *__restrict__ dz,
                                                      float *__restrict__ part) {
  __shared__ double lds[BS / 64];
  const int co = blockIdx.x, b = blockIdx.y;
  const int64_t q0 = (int64_t)b * chunk, q1 = min(P, q0 + chunk);
  const uint16_t *row = dz + (size_t)co * P;
  double v = 0;
#pragma unroll 8
  for (int64_t q = q0 + threadIdx.x; q < q1; q += BS) v += bf2f(row[q]);
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + co] = (float)s;
}

// wrot[ci][ky][kx][co] = w[co][2-ky][2-kx][ci]: the data gradient is the
// forward convolution of dz with these weights.
__global__ void __launch_bounds__(BS) rot_kernel(int cin, int cout, const uint16_t *__restrict__ w,
                                                uint16_t *__restrict__ wrot) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= (int64_t)cin * cout * 9) return;
  const int ci = (int)(i % cin), tap = (int)((i / cin) % 9), co = (int)(i / (9 * (int64_t)cin));
  wrot[((size_t)ci * 9 + (8 - tap)) * cout + co] = w[i];
}

// Every layer of a table in one launch: the turned, transposed layout of
// rot_kernel at wrot + off[l] from layer l's weights at w + off[l] (layout
// [cout][3][3][cin]).  Thread i writes element k of layer l's output (so the
// stores are contiguous and the scattered accesses are the reads); it finds
// its layer by scanning the prefix counts (at most kRotLayers entries).
constexpr int kRotLayers = 32;
struct RotTable {
  int n;
  int cin[kRotLayers], cout[kRotLayers];
  int64_t off[kRotLayers], first[kRotLayers + 1];
};

__global__ void __launch_bounds__(BS) rot_all_kernel(const RotTable t, const uint16_t *__restrict__ w,
                                                    uint16_t *__restrict__ wrot) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= t.first[t.n]) return;
  int l = 0;
  while (l + 1 < t.n && i >= t.first[l + 1]) ++l;
  const int64_t k = i - t.first[l];
  const int cin = t.cin[l], cout = t.cout[l];
  const int co = (int)(k % cout), rtap = (int)((k / cout) % 9), ci = (int)(k / (9 * (int64_t)cout));
  wrot[t.off[l] + k] = w[t.off[l] + ((int64_t)co * 9 + (8 - rtap)) * cin + ci];
}

__global__ void __launch_bounds__(BS) relu_kernel(int64_t n, const float *__restrict__ z, uint16_t *__restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) a[i] = f2bf(fmaxf(z[i], 0.f));
}

__global__ void __launch_bounds__(BS) relu_back_kernel(int64_t n, const uint16_t *__restrict__ a,
                                                      const float *__restrict__ da, uint16_t *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) dz[i] = f2bf(bf2f(a[i]) > 0.f ? da[i] : 0.f);
}

// The same on eight elements per thread (count % 8 == 0, 16-byte aligned).
__global__ void __launch_bounds__(BS) relu_back8_kernel(int64_t n8, const uint4 *__restrict__ a,
                                                       const float4 *__restrict__ da, uint4 *__restrict__ dz) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n8) return;
  const uint4 av = a[i];
  const float4 d0 = da[2 * i], d1 = da[2 * i + 1];
  const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
  const float dv[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint16_t lo = f2bf(bf2f((uint16_t)(aw[k] & 0xffffu)) > 0.f ? dv[2 * k] : 0.f);
    const uint16_t hi = f2bf(bf2f((uint16_t)(aw[k] >> 16)) > 0.f ? dv[2 * k + 1] : 0.f);
    o[k] = (uint32_t)lo | ((uint32_t)hi << 16);
  }
  dz[i] = uint4{o[0], o[1], o[2], o[3]};
}

__global__ void __launch_bounds__(BS) to_bf16_kernel(int64_t n, const float *__restrict__ x, uint16_t *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

__global__ void __launch_bounds__(BS) from_bf16_kernel(int64_t n, const uint16_t *__restrict__ x, float *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) y[i] = bf2f(x[i]);
}

// y[plane][i][j] = mean of x[plane][2i..2i+1][2j..2j+1]
__global__ void __launch_bounds__(BS) pool2_kernel(int64_t planes, int h, int w, const uint16_t *__restrict__ x,
                                                  uint16_t *__restrict__ y) {
  const int ho = h / 2, wo = w / 2;
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * ho * wo) return;
  const int64_t pl = i / ((int64_t)ho * wo);
  const int r = (int)(i % ((int64_t)ho * wo)), yi = r / wo, xi = r - yi * wo;
  const uint16_t *b = x + (size_t)pl * h * w + (size_t)(2 * yi) * w + 2 * xi;
  y[i] = f2bf(0.25f * (bf2f(b[0]) + bf2f(b[1]) + bf2f(b[w]) + bf2f(b[w + 1])));
}

__global__ void __launch_bounds__(BS) pool2_back_kernel(int64_t planes, int h, int w, const float *__restrict__ dy,
                                                       float *__restrict__ dx) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * h * w) return;
  const int64_t pl = i / ((int64_t)h * w);
  const int r = (int)(i % ((int64_t)h * w)), yi = r / w, xi = r - yi * w;
  dx[i] = 0.25f * dy[(size_t)pl * (h / 2) * (w / 2) + (size_t)(yi / 2) * (w / 2) + xi / 2];
}

// y[plane][2i+a][2j+b] = x[plane][i][j]
__global__ void __launch_bounds__(BS) up2_kernel(int64_t planes, int h, int w, const uint16_t *__restrict__ x,
                                                uint16_t *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * 4 * h * w) return;
  const int64_t pl = i / (4 * (int64_t)h * w);
  const int r = (int)(i % (4 * (int64_t)h * w)), yi = r / (2 * w), xi = r - yi * (2 * w);
  y[i] = x[(size_t)pl * h * w + (size_t)(yi / 2) * w + xi / 2];
}

// Vector forms for w % 4 == 0: pool2_back writes four outputs of each of
// two rows from two gradients; up2 copies four inputs to eight outputs of
// each of two rows (16-byte stores).
__global__ void __launch_bounds__(BS) pool2_back4_kernel(int64_t planes, int h, int w, const float *__restrict__ dy,
                                                        float *__restrict__ dx) {
  const int wq = w / 4, ho = h / 2;
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * ho * wq) return;
  const int64_t pl = i / ((int64_t)ho * wq);
  const int r = (int)(i % ((int64_t)ho * wq)), yo = r / wq, xq = r - yo * wq;
  const float2 g = *(const float2 *)(dy + (size_t)pl * ho * (w / 2) + (size_t)yo * (w / 2) + 2 * xq);
  const float4 v = {0.25f * g.x, 0.25f * g.x, 0.25f * g.y, 0.25f * g.y};
  float *b = dx + (size_t)pl * h * w + (size_t)(2 * yo) * w + 4 * xq;
  *(float4 *)b = v;
  *(float4 *)(b + w) = v;
}

__global__ void __launch_bounds__(BS) up2x4_kernel(int64_t planes, int h, int w, const uint16_t *__restrict__ x,
                                                  uint16_t *__restrict__ y) {
  const int wq = w / 4;
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * h * wq) return;
  const int64_t pl = i / ((int64_t)h * wq);
  const int r = (int)(i % ((int64_t)h * wq)), yi = r / wq, xq = r - yi * wq;
  const uint2 v = *(const uint2 *)(x + (size_t)pl * h * w + (size_t)yi * w + 4 * xq);
  const uint32_t e[4] = {v.x & 0xffffu, v.x >> 16, v.y & 0xffffu, v.y >> 16};
  const uint4 o = {e[0] | (e[0] << 16), e[1] | (e[1] << 16), e[2] | (e[2] << 16), e[3] | (e[3] << 16)};
  uint16_t *b = y + (size_t)pl * 4 * h * w + (size_t)(2 * yi) * (2 * w) + 8 * xq;
  *(uint4 *)b = o;
  *(uint4 *)(b + 2 * w) = o;
}

// up2_back on two outputs per thread (w % 2 == 0): two 16-byte row reads.
__global__ void __launch_bounds__(BS) up2_back2_kernel(int64_t planes, int h, int w, const float *__restrict__ dy,
                                                      float *__restrict__ dx) {
  const int wh = w / 2;
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * h * wh) return;
  const int64_t pl = i / ((int64_t)h * wh);
  const int r = (int)(i % ((int64_t)h * wh)), yi = r / wh, xh = r - yi * wh;
  const float *b = dy + (size_t)pl * 4 * h * w + (size_t)(2 * yi) * (2 * w) + 4 * xh;
  const float4 u = *(const float4 *)b, d = *(const float4 *)(b + 2 * w);
  *(float2 *)(dx + (size_t)pl * h * w + (size_t)yi * w + 2 * xh) = float2{u.x + u.y + d.x + d.y, u.z + u.w + d.z + d.w};
}

__global__ void __launch_bounds__(BS) up2_back_kernel(int64_t planes, int h, int w, const float *__restrict__ dy,
                                                     float *__restrict__ dx) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= planes * h * w) return;
  const int64_t pl = i / ((int64_t)h * w);
  const int r = (int)(i % ((int64_t)h * w)), yi = r / w, xi = r - yi * w;
  const float *b = dy + (size_t)pl * 4 * h * w + (size_t)(2 * yi) * (2 * w) + 2 * xi;
  dx[i] = b[0] + b[1] + b[2 * w] + b[2 * w + 1];
}

__global__ void __launch_bounds__(BS) adam_kernel(int64_t n, float *__restrict__ p, float *__restrict__ m,
                                                 float *__restrict__ v, const float *__restrict__ g,
                                                 uint16_t *__restrict__ pb, float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = f2bf(pi);
}

__global__ void __launch_bounds__(BS) axpy_kernel(int64_t n, float a, const float *__restrict__ x, float *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

__global__ void __launch_bounds__(BS) axpy4_kernel(int64_t n4, float a, const float4 *__restrict__ x,
                                                  float4 *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= n4) return;
  const float4 u = x[i];
  float4 v = y[i];
  v.x += a * u.x;
  v.y += a * u.y;
  v.z += a * u.z;
  v.w += a * u.w;
  y[i] = v;
}

// grad = 2 (pred - target) * scale; partial sums of (pred - target)^2
__global__ void __launch_bounds__(BS) mse_kernel(int64_t n, const float *__restrict__ pred,
                                                const float *__restrict__ target, float scale,
                                                float *__restrict__ grad, double *__restrict__ part) {
  __shared__ double lds[BS / 64];
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  double e2 = 0;
  if (i < n) {
    const float d = pred[i] - target[i];
    if (grad) grad[i] = 2.f * d * scale;
    e2 = (double)d * d;
  }
  const double s = block_sum(e2, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(BS) sum_kernel(const double *__restrict__ part, int nb, double *__restrict__ out) {
  __shared__ double lds[BS / 64];
  double v = 0;
  for (int b = threadIdx.x; b < nb; b += BS) v += part[b];
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) out[0] = s;
}

// out[n] = bl + sum_c wl[c] mean_p a[c][n][p]; one workgroup per image.
__global__ void __launch_bounds__(BS) gap_linear_kernel(int nimg, int c, int hw, const uint16_t *__restrict__ a,
                                                       const float *__restrict__ wl, const float *__restrict__ bl,
                                                       float *__restrict__ out) {
  __shared__ double lds[BS / 64];
  const int n = blockIdx.x;
  double v = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)c * hw; i += BS) {
    const int ch = (int)(i / hw), p = (int)(i - (int64_t)ch * hw);
    v += (double)wl[ch] * bf2f(a[((size_t)ch * nimg + n) * hw + p]);
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) out[n] = (float)(s / hw + bl[0]);
}

// da[c][n][p] = dout[n] wl[c] / hw
__global__ void __launch_bounds__(BS) gap_linear_back_a_kernel(int nimg, int c, int hw, const float *__restrict__ dout,
                                                              const float *__restrict__ wl, float *__restrict__ da) {
  const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (i >= (int64_t)c * nimg * hw) return;
  const int64_t cn = i / hw;
  const int ch = (int)(cn / nimg), n = (int)(cn - (int64_t)ch * nimg);
  da[i] = dout[n] * wl[ch] / (float)hw;
}

// dwl[c] = sum_n dout[n] mean_p a[c][n][p]; dbl = sum_n dout[n].  One workgroup per channel (+1 for the bias).
// The same for hw % 64 == 0: one 1024-thread workgroup per image, wavefront
// wv takes channels wv, wv + 16, ..., its lanes pixels lane + 64 k (FP64
// sums, a fixed order).
__global__ void __launch_bounds__(1024) gap_linear64_kernel(int nimg, int c, int hw, const uint16_t *__restrict__ a,
                                                           const float *__restrict__ wl, const float *__restrict__ bl,
                                                           float *__restrict__ out) {
  __shared__ double lds[16];
  const int n = blockIdx.x, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double v = 0;
  for (int ch = wv; ch < c; ch += 16) {
    const uint16_t *row = a + ((size_t)ch * nimg + n) * hw;
    double sp = 0;
#pragma unroll 4
    for (int p = lane; p < hw; p += 64) sp += bf2f(row[p]);
    v += (double)wl[ch] * sp;
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < 16; ++k) s += lds[k];
    out[n] = (float)(s / hw + bl[0]);
  }
}

__global__ void __launch_bounds__(BS) gap_linear_back_w_kernel(int nimg, int c, int hw, const uint16_t *__restrict__ a,
                                                              const float *__restrict__ dout, float *__restrict__ dwl,
                                                              float *__restrict__ dbl) {
  __shared__ double lds[BS / 64];
  const int ch = blockIdx.x;
  double v = 0;
  if (ch < c) {
    for (int64_t i = threadIdx.x; i < (int64_t)nimg * hw; i += BS)
      v += (double)dout[i / hw] * bf2f(a[(size_t)ch * nimg * hw + i]);
  } else {
    for (int n = threadIdx.x; n < nimg; n += BS) v += dout[n];
  }
  const double s = block_sum(v, lds);
  if (threadIdx.x == 0) {
    if (ch < c) dwl[ch] = (float)(s / hw);
    else dbl[0] = (float)s;
  }
}

int nb_of(int64_t n) { return (int)((n + BS - 1) / BS); }
bool aligned(const void *p, uintptr_t b) { return ((uintptr_t)p & (b - 1)) == 0; }

thread_local std::string g_err;

template <typename F>
fdtd_status nguard(F &&f) {
  try {
    f();
    return FDTD_OK;
  } catch (const Error &e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::exception &e) {
    g_err = e.what();
    return FDTD_EDEVICE;
  }
}

void need(bool ok) {
  if (!ok) throw Error{FDTD_EINVAL, "invalid sizes or missing pointer"};
}


}  // namespace

extern "C" {

fdtd_status fdtd_nn_conv3x3(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *x,
                            const uint16_t *wt, const float *bias, float *z, uint16_t *a, void *stream) {
  return nguard([&] {
    need(n > 0 && n <= 65535 && cin > 0 && cout > 0 && h > 0 && w > 0 && x && wt && (z || a));
    launch_conv(n, cin, cout, h, w, x, wt, bias, z, a, nullptr, (hipStream_t)stream);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_conv3x3_dgrad(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *dz,
                                  const uint16_t *wt, uint16_t *wrot, float *dx, void *stream) {
  return nguard([&] {
    need(n > 0 && n <= 65535 && cin > 0 && cout > 0 && h > 0 && w > 0 && dz && wrot && dx);
    hipStream_t s = (hipStream_t)stream;
    if (wt) hipLaunchKernelGGL(rot_kernel, dim3(nb_of((int64_t)cin * cout * 9)), dim3(BS), 0, s, cin, cout, wt, wrot);
    launch_conv(n, cout, cin, h, w, dz, wrot, nullptr, dx, nullptr, nullptr, s);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_conv3x3_dgrad_relu(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *dz,
                                       const uint16_t *wt, uint16_t *wrot, const uint16_t *a, uint16_t *dza,
                                       void *stream) {
  return nguard([&] {
    need(n > 0 && n <= 65535 && cin > 0 && cout > 0 && h > 0 && w > 0 && dz && wrot && a && dza);
    hipStream_t s = (hipStream_t)stream;
    if (wt) hipLaunchKernelGGL(rot_kernel, dim3(nb_of((int64_t)cin * cout * 9)), dim3(BS), 0, s, cin, cout, wt, wrot);
    launch_conv(n, cout, cin, h, w, dz, wrot, nullptr, nullptr, dza, a, s);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_rot_weights(int32_t nlayers, const int32_t *cin, const int32_t *cout, const int64_t *off,
                                const uint16_t *w, uint16_t *wrot, void *stream) {
  return nguard([&] {
    need(nlayers >= 1 && nlayers <= kRotLayers && cin && cout && off && w && wrot);
    RotTable t{};
    t.n = nlayers;
    t.first[0] = 0;
    for (int l = 0; l < nlayers; ++l) {
      need(cin[l] > 0 && cout[l] > 0 && off[l] >= 0);
      t.cin[l] = cin[l];
      t.cout[l] = cout[l];
      t.off[l] = off[l];
      t.first[l + 1] = t.first[l] + (int64_t)cin[l] * cout[l] * 9;
    }
    need(t.first[nlayers] <= (int64_t)INT32_MAX * BS);
    hipLaunchKernelGGL(rot_all_kernel, dim3(nb_of(t.first[nlayers])), dim3(BS), 0, (hipStream_t)stream, t, w, wrot);
    FDTD_HIP(hipGetLastError());
  });
}

int64_t fdtd_nn_wgrad_work(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w) {
  if (n <= 0 || cin <= 0 || cout <= 0 || h <= 0 || w <= 0) return 0;
  const int64_t P = (int64_t)n * h * w, splits = wgrad_plan(n, cin, cout, h, w).splits;
  // tiled: splits rows of cout * cin * 9 weight and cout bias sums; generic:
  // the weight rows, then bias_ranges(P) rows of cout bias sums
  return splits * cout * cin * 9 + std::max(splits, bias_ranges(P)) * cout;
}

}  // extern "C"

// Scratch of the allocation-free weight gradient: one array per device,
// held until the process ends (64 MiB: the largest workspace the split plan
// asks for, about 768 partial sums of a 64 x 32 x 9 block, is 54 MiB).  In
// host code `scratch` names a host-side stand-in, never the device memory:
// kernels get the address hipGetSymbolAddress returns on each device.
static constexpr int64_t kScratchFloats = int64_t(16) << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

// The weight and bias gradients with partial sums in `work` (at least
// fdtd_nn_wgrad_work floats; every slot the reductions read is written first).
void wgrad_run(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *x, const uint16_t *dz,
               float *dw, float *db, float *work, hipStream_t s) {
    const int K = cin * 9;
    const int64_t P = (int64_t)n * h * w;
    const WgradPlan pl = wgrad_plan(n, cin, cout, h, w);
    const int64_t m = (int64_t)cout * K;
    if (pl.c1) {
      // partial rows [split][m weight sums | cout bias sums]
      const int64_t stride = m + cout;
      hipLaunchKernelGGL(conv1_wgrad_kernel, dim3(pl.splits), dim3(BS), 0, s, n, cout, h, w, x, dz, work, stride,
                         pl.chunk, db ? work + m : nullptr);
      if (db && db == dw + m) {
        launch_split_sum(work, pl.splits, stride, m + cout, dw, s);
      } else {
        launch_split_sum(work, pl.splits, stride, m, dw, s);
        if (db) launch_split_sum(work + m, pl.splits, stride, cout, db, s);
      }
    } else if (pl.tiled && ((uintptr_t)dz & 15) == 0 && ((uintptr_t)x & 15) == 0) {
      // partial rows [split][m weight sums | cout bias sums]
      const int64_t stride = m + cout;
      const int ct = wgrad_ct(cout);
      const dim3 g((cout + ct - 1) / ct, cin / 32, pl.splits);
      float *bp = db ? work + m : nullptr;
      if (ct == 32)
        hipLaunchKernelGGL(conv_wgrad_mfma_kernel<32>, g, dim3(BS), 0, s, n, cin, cout, h, w, x, dz, work, stride,
                           pl.chunk, bp);
      else
        hipLaunchKernelGGL(conv_wgrad_mfma_kernel<64>, g, dim3(BS), 0, s, n, cin, cout, h, w, x, dz, work, stride,
                           pl.chunk, bp);
      if (db && db == dw + m) {  // contiguous weight and bias gradients: one reduction
        launch_split_sum(work, pl.splits, stride, m + cout, dw, s);
      } else {
        launch_split_sum(work, pl.splits, stride, m, dw, s);
        if (db) launch_split_sum(work + m, pl.splits, stride, cout, db, s);
      }
    } else {
      // generic kernel, at most as many pixel ranges as the plan has partial sums
      int64_t chunk = (P + pl.splits - 1) / pl.splits;
      chunk = (chunk + TK - 1) / TK * TK;
      const int S = (int)((P + chunk - 1) / chunk);
      const dim3 g((K + TN - 1) / TN, (cout + TM - 1) / TM, S);
      hipLaunchKernelGGL(conv_wgrad_kernel, g, dim3(BS), 0, s, n, cin, cout, h, w, x, dz, work, (int)chunk);
      launch_split_sum(work, S, m, m, dw, s);
      if (db) {
        float *pb = work + (size_t)pl.splits * m;
        const int64_t nr = bias_ranges(P), bchunk = (P + nr - 1) / nr;
        hipLaunchKernelGGL(bias_grad_kernel, dim3(cout, (unsigned)nr), dim3(BS), 0, s, P, bchunk, dz, pb);
        launch_split_sum(pb, (int)nr, cout, cout, db, s);
      }
    }
    FDTD_HIP(hipGetLastError());
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
float *scratch_on_current_device() {
  int dev = 0;
  FDTD_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<int, float *> ptrs;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ptrs.find(dev);
  if (it != ptrs.end()) return it->second;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error{FDTD_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e)};
  }
  ptrs[dev] = static_cast<float *>(p);
  return ptrs[dev];
}

}  // namespace

extern "C" {

fdtd_status fdtd_nn_conv3x3_wgrad(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w, const uint16_t *x,
                                  const uint16_t *dz, float *dw, float *db, float *work, void *stream) {
  return nguard([&] {
    need(n > 0 && cin > 0 && cout > 0 && h > 0 && w > 0 && x && dz && dw && work);
    wgrad_run(n, cin, cout, h, w, x, dz, dw, db, work, (hipStream_t)stream);
  });
}

fdtd_status fdtd_nn_conv3x3_wgrad_noalloc(int32_t n, int32_t cin, int32_t cout, int32_t h, int32_t w,
                                          const uint16_t *x, const uint16_t *dz, float *dw, float *db, void *stream) {
  return nguard([&] {
    need(n > 0 && cin > 0 && cout > 0 && h > 0 && w > 0 && x && dz && dw);
    const int64_t want = fdtd_nn_wgrad_work(n, cin, cout, h, w);
    if (want > kScratchFloats)
      throw Error{FDTD_EINVAL, "weight gradient needs " + std::to_string(want) + " floats of scratch; the static array "
                               "holds " + std::to_string(kScratchFloats) + " (use fdtd_nn_conv3x3_wgrad with a workspace)"};
    wgrad_run(n, cin, cout, h, w, x, dz, dw, db, scratch_on_current_device(), (hipStream_t)stream);
  });
}

fdtd_status fdtd_nn_relu_bf16(int64_t count, const float *z, uint16_t *a, void *stream) {
  return nguard([&] {
    need(count > 0 && z && a);
    hipLaunchKernelGGL(relu_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, z, a);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_relu_bf16_backward(int64_t count, const uint16_t *a, const float *da, uint16_t *dz,
                                       void *stream) {
  return nguard([&] {
    need(count > 0 && a && da && dz);
    if (count % 8 == 0 && aligned(a, 16) && aligned(da, 16) && aligned(dz, 16))
      hipLaunchKernelGGL(relu_back8_kernel, dim3(nb_of(count / 8)), dim3(BS), 0, (hipStream_t)stream, count / 8,
                         (const uint4 *)a, (const float4 *)da, (uint4 *)dz);
    else
      hipLaunchKernelGGL(relu_back_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, a, da, dz);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_to_bf16(int64_t count, const float *x, uint16_t *y, void *stream) {
  return nguard([&] {
    need(count > 0 && x && y);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, x, y);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_from_bf16(int64_t count, const uint16_t *x, float *y, void *stream) {
  return nguard([&] {
    need(count > 0 && x && y);
    hipLaunchKernelGGL(from_bf16_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, x, y);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_pool2(int64_t planes, int32_t h, int32_t w, const uint16_t *x, uint16_t *y, void *stream) {
  return nguard([&] {
    need(planes > 0 && h > 1 && w > 1 && h % 2 == 0 && w % 2 == 0 && x && y);
    hipLaunchKernelGGL(pool2_kernel, dim3(nb_of(planes * (h / 2) * (w / 2))), dim3(BS), 0, (hipStream_t)stream,
                       planes, h, w, x, y);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_pool2_backward(int64_t planes, int32_t h, int32_t w, const float *dy, float *dx, void *stream) {
  return nguard([&] {
    need(planes > 0 && h > 1 && w > 1 && h % 2 == 0 && w % 2 == 0 && dy && dx);
    if (w % 4 == 0 && aligned(dy, 8) && aligned(dx, 16))
      hipLaunchKernelGGL(pool2_back4_kernel, dim3(nb_of(planes * (h / 2) * (w / 4))), dim3(BS), 0,
                         (hipStream_t)stream, planes, h, w, dy, dx);
    else
      hipLaunchKernelGGL(pool2_back_kernel, dim3(nb_of(planes * h * w)), dim3(BS), 0, (hipStream_t)stream, planes, h,
                         w, dy, dx);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_up2(int64_t planes, int32_t h, int32_t w, const uint16_t *x, uint16_t *y, void *stream) {
  return nguard([&] {
    need(planes > 0 && h > 0 && w > 0 && x && y);
    if (w % 4 == 0 && aligned(x, 8) && aligned(y, 16))
      hipLaunchKernelGGL(up2x4_kernel, dim3(nb_of(planes * h * (w / 4))), dim3(BS), 0, (hipStream_t)stream, planes, h,
                         w, x, y);
    else
      hipLaunchKernelGGL(up2_kernel, dim3(nb_of(planes * 4 * h * w)), dim3(BS), 0, (hipStream_t)stream, planes, h, w,
                         x, y);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_up2_backward(int64_t planes, int32_t h, int32_t w, const float *dy, float *dx, void *stream) {
  return nguard([&] {
    need(planes > 0 && h > 0 && w > 0 && dy && dx);
    if (w % 2 == 0 && aligned(dy, 16) && aligned(dx, 8))
      hipLaunchKernelGGL(up2_back2_kernel, dim3(nb_of(planes * h * (w / 2))), dim3(BS), 0, (hipStream_t)stream,
                         planes, h, w, dy, dx);
    else
      hipLaunchKernelGGL(up2_back_kernel, dim3(nb_of(planes * h * w)), dim3(BS), 0, (hipStream_t)stream, planes, h,
                         w, dy, dx);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_adam(int64_t count, float *p, float *m, float *v, const float *g, uint16_t *pb, float lr,
                         float beta1, float beta2, float eps, int32_t t, void *stream) {
  return nguard([&] {
    need(count > 0 && p && m && v && g && t >= 1);
    const float c1 = 1.f - std::pow(beta1, (float)t), c2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, p, m, v, g, pb, lr,
                       beta1, beta2, eps, c1, c2);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_axpy(int64_t count, float a, const float *x, float *y, void *stream) {
  return nguard([&] {
    need(count > 0 && x && y);
    if (count % 4 == 0 && aligned(x, 16) && aligned(y, 16))
      hipLaunchKernelGGL(axpy4_kernel, dim3(nb_of(count / 4)), dim3(BS), 0, (hipStream_t)stream, count / 4, a,
                         (const float4 *)x, (float4 *)y);
    else
      hipLaunchKernelGGL(axpy_kernel, dim3(nb_of(count)), dim3(BS), 0, (hipStream_t)stream, count, a, x, y);
    FDTD_HIP(hipGetLastError());
  });
}

int64_t fdtd_nn_mse_work(int64_t count) { return count > 0 ? nb_of(count) : 0; }

fdtd_status fdtd_nn_mse(int64_t count, const float *pred, const float *target, float scale, float *grad,
                        double *work, double *sum_sq, void *stream) {
  return nguard([&] {
    need(count > 0 && pred && target && work && sum_sq);
    hipStream_t s = (hipStream_t)stream;
    const int nb = nb_of(count);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(BS), 0, s, count, pred, target, scale, grad, work);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(BS), 0, s, work, nb, sum_sq);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_gap_linear(int32_t n, int32_t c, int32_t hw, const uint16_t *a, const float *wl, const float *bl,
                               float *out, void *stream) {
  return nguard([&] {
    need(n > 0 && c > 0 && hw > 0 && a && wl && bl && out);
    if (hw % 64 == 0)
      hipLaunchKernelGGL(gap_linear64_kernel, dim3(n), dim3(1024), 0, (hipStream_t)stream, n, c, hw, a, wl, bl, out);
    else
      hipLaunchKernelGGL(gap_linear_kernel, dim3(n), dim3(BS), 0, (hipStream_t)stream, n, c, hw, a, wl, bl, out);
    FDTD_HIP(hipGetLastError());
  });
}

fdtd_status fdtd_nn_gap_linear_backward(int32_t n, int32_t c, int32_t hw, const uint16_t *a, const float *wl,
                                        const float *dout, float *da, float *dwl, float *dbl, void *stream) {
  return nguard([&] {
    need(n > 0 && c > 0 && hw > 0 && a && wl && dout && da && dwl && dbl);
    hipStream_t s = (hipStream_t)stream;
    const int64_t total = (int64_t)n * c * hw;
    hipLaunchKernelGGL(gap_linear_back_a_kernel, dim3(nb_of(total)), dim3(BS), 0, s, n, c, hw, dout, wl, da);
    hipLaunchKernelGGL(gap_linear_back_w_kernel, dim3(c + 1), dim3(BS), 0, s, n, c, hw, a, dout, dwl, dbl);
    FDTD_HIP(hipGetLastError());
  });
}

const char *fdtd_nn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
