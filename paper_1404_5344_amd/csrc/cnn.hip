// Warm-start network: six 3x3 convolutions (1 -> 32, 4 x 32 -> 32, 32 -> 1), zero "same"
// padding, ReLU after the first five, input log f - 4.5, output w0 = log f + net.  Hand-written
// forward, backward-data, backward-weight, loss and Adam kernels.  Weights are BF16 (the
// FP32 master weights rounded to BF16 after every Adam step); activations are FP32 NCHW planes.
// The 32 -> 32 layers run on the BF16 matrix cores as implicit GEMMs (forward, backward-data and
// backward-weight), every FP32 activation or gradient split into three BF16 parts, FP32 accumulation;
// the 1 -> 32 and 32 -> 1 layers on the VALU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/foe.h"
#include "device_math.hpp"

namespace cnn {

constexpr int NL = 6;
constexpr int CIN[NL] = {1, 32, 32, 32, 32, 32};
constexpr int COUT[NL] = {32, 32, 32, 32, 32, 1};
constexpr float SHIFT = 4.5f;
constexpr int TS = 16;  // spatial tile of the convolution kernels

__host__ __device__ constexpr int layer_params(int l) { return COUT[l] * CIN[l] * 9 + COUT[l]; }
__host__ constexpr int total_params() {
  int n = 0;
  for (int l = 0; l < NL; ++l) n += layer_params(l);
  return n;
}

// The tile of block b of a 1-D grid of 8 * per blocks over ntiles tiles (images, tile rows, tile columns,
// row-major): blocks are dealt to the 8 XCDs in turn, so XCD b % 8 takes the consecutive tiles
// (b % 8) per .. (b % 8 + 1) per - 1, and tiles that share halo lines share one L2.  False when the
// block has no tile.
__device__ __forceinline__ bool xcd_tile(int H, int W, int n_img, int* x0, int* y0, int* n) {
  const int tx = (W + TS - 1) / TS, ty = (H + TS - 1) / TS, ntiles = tx * ty * n_img;
  const int per = (ntiles + 7) / 8;
  const int t = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (t >= ntiles) return false;
  *n = t / (tx * ty);
  const int r = t - *n * (tx * ty);
  *y0 = (r / tx) * TS;
  *x0 = (r % tx) * TS;
  return true;
}

// out[n][co][p] = act(bias[co] + sum_ci sum_t wt[ci][t][co] in[n][ci][p + off_t]) * (mask[n][co][p] > 0),
// act = ReLU when relu != 0; bias and mask nullable; zero padding.  wt (CI 9 CO values) is staged in
// LDS and read as block-wide broadcasts.
// One 16 x 16 tile per block (xcd_tile).
template <int CI, int CO, int CICH>
__global__ __launch_bounds__(256) void conv3_kernel(const float* __restrict__ in, const float* __restrict__ wt,
                                                    const float* __restrict__ bias, float* __restrict__ out,
                                                    const float* __restrict__ mask, int H, int W, int n_img,
                                                    int relu) {
  __shared__ float tile[CICH][TS + 2][TS + 2];
  __shared__ __attribute__((aligned(16))) float w[CI * 9 * CO];
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  int x0, y0, n;
  if (!xcd_tile(H, W, n_img, &x0, &y0, &n)) return;
  const size_t plane = (size_t)H * W;
  const float* inb = in + (size_t)n * CI * plane;
  for (int i = threadIdx.x; i < CI * 9 * CO; i += 256) w[i] = wt[i];
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias ? bias[co] : 0.0f;
  // the loads of chunk c0 + CICH are issued before the arithmetic on chunk c0 and wait in registers;
  // branch-free (clamped positions, zero off the image)
  constexpr int ITEMS = CICH * (TS + 2) * (TS + 2), PER = (ITEMS + 255) / 256;
  float v[PER];
  auto fetch = [&](int c0) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      const int ci = min(i / ((TS + 2) * (TS + 2)), CICH - 1), r = (i / (TS + 2)) % (TS + 2), c = i % (TS + 2);
      const int y = y0 + r - 1, x = x0 + c - 1;
      const bool ok = i < ITEMS && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
      const float a = inb[(c0 + ci) * plane + (size_t)(min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1))];
      v[k] = ok ? a : 0.0f;
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < CI; c0 += CICH) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < ITEMS) (&tile[0][0][0])[i] = v[k];
    }
    __syncthreads();
    if (c0 + CICH < CI) fetch(c0 + CICH);
    auto tap = [&](int ci, int t) {
      const float v = tile[ci][ty + t / 3][tx + t % 3];
      const float* wr = w + ((c0 + ci) * 9 + t) * CO;
#pragma unroll
      for (int co = 0; co < CO; ++co) acc[co] = fmaf(wr[co], v, acc[co]);
    };
#pragma unroll 1
    for (int ci = 0; ci < CICH; ++ci) {
      if constexpr (CO > 8) {   // the taps one at a time: CO weights in registers, not 9 CO
#pragma unroll 1
        for (int t = 0; t < 9; ++t) tap(ci, t);
      } else {
#pragma unroll
        for (int t = 0; t < 9; ++t) tap(ci, t);
      }
    }
    __syncthreads();
  }
  const int x = x0 + tx, y = y0 + ty;
  if (x >= W || y >= H) return;
  float* ob = out + (size_t)n * CO * plane + (size_t)y * W + x;
  const float* mb = mask ? mask + (size_t)n * CO * plane + (size_t)y * W + x : nullptr;
#pragma unroll
  for (int co = 0; co < CO; ++co) {
    float v = relu ? fmaxf(acc[co], 0.0f) : acc[co];
    if (mb) v = mb[co * plane] > 0.0f ? v : 0.0f;
    ob[co * plane] = v;
  }
}

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// A 32 -> 32 layer on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16): per 3x3 tap t an implicit GEMM
//   out[co][p] += sum_ci wt[ci][t][co] in[ci][p + off_t],
// M = 16 output channels, N = 16 pixels (one tile row), K = the 32 input channels.  The taps are BF16
// values (exact); each FP32 input is split into three BF16 numbers, in = s0 + s1 + s2 with s0 = bf16(in),
// s1 = bf16(in - s0), s2 = bf16(in - s0 - s1) (the rest is below 2^-27 |in|, under FP32 rounding), and all
// three are multiplied, the products exact and summed in FP32.  One 16 x 16 tile per block (xcd_tile), its
// input (with the 1-pixel halo) staged channel-last in LDS, 40 halves per pixel (80 B: the 8 channels of a
// lane start on 16 bytes, and 16 consecutive pixels cover the 64 banks once).  Wave w takes tile rows
// 4w .. 4w + 3, both channel blocks; act, bias and mask as conv3_kernel.  amat: the A operands of the layer
// (mfma_taps_kernel).
__global__ __launch_bounds__(256) void conv32_mfma_kernel(const float* __restrict__ in, const uint4* __restrict__ amat,
                                                          const float* __restrict__ bias, float* __restrict__ out,
                                                          const float* __restrict__ mask, int H, int W, int n_img,
                                                          int relu) {
  constexpr int C = 32, TP = TS + 2, PW = 40;
  __shared__ __attribute__((aligned(16))) unsigned ts[3][TP * TP * PW / 2];   // the three BF16 parts
  const int tid = threadIdx.x, lane = tid & 63, ln = lane & 15, kg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int x0, y0, n;
  if (!xcd_tile(H, W, n_img, &x0, &y0, &n)) return;
  const size_t plane = (size_t)H * W;
  const unsigned pl = (unsigned)plane;
  // one channel pair of one pixel per item, every load in flight before the first LDS store; branch-free:
  // each item loads from a clamped position (32-bit byte offsets in the image's 32 planes, which the host
  // keeps below 2^32) and keeps zero off the image
  constexpr int ITEMS = (C / 2) * TP * TP, PER = (ITEMS + 255) / 256;
  float v0[PER], v1[PER];
  {
    const char* inb = reinterpret_cast<const char*>(in + (size_t)n * C * plane);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = tid + 256 * k;
      const int cp = min(i / (TP * TP), C / 2 - 1), pix = i - (i / (TP * TP)) * (TP * TP);
      const int r = pix / TP, c = pix - r * TP;
      const int y = y0 + r - 1, x = x0 + c - 1;
      const bool ok = i < ITEMS && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
      const unsigned off =
          4u * ((unsigned)(2 * cp) * pl + (unsigned)(min(max(y, 0), H - 1) * W + min(max(x, 0), W - 1)));
      const float a = *reinterpret_cast<const float*>(inb + off);
      const float b = *reinterpret_cast<const float*>(inb + off + 4u * pl);
      v0[k] = ok ? a : 0.0f;
      v1[k] = ok ? b : 0.0f;
    }
  }
  // A operands: lane (m, k) holds wt[8k + i][t][16 mb + m], i = 0..7
  bf16x8 A[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) A[t][mb] = __builtin_bit_cast(bf16x8, amat[(t * 2 + mb) * 64 + lane]);
  // stage, as words of two BF16 (the even channel low)
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = tid + 256 * k;
    if (i >= ITEMS) break;
    const int cp = i / (TP * TP), pix = i - cp * (TP * TP);
    float a0 = v0[k], a1 = v1[k];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const __bf16 h0 = (__bf16)a0, h1 = (__bf16)a1;
      ts[q][pix * (PW / 2) + cp] = (unsigned)__builtin_bit_cast(unsigned short, h0) |
                                   ((unsigned)__builtin_bit_cast(unsigned short, h1) << 16);
      a0 -= (float)h0;   // exact: the remainder of a BF16 rounding of an FP32 number
      a1 -= (float)h1;
    }
  }
  float bv[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[mb][j] = bias ? bias[16 * mb + 4 * kg + j] : 0.0f;
  __syncthreads();
  const int x = x0 + ln;
#pragma unroll 1
  for (int rr = 0; rr < 4; ++rr) {
    const int row = wave * 4 + rr;
    floatx4 acc[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      // B operand: lane (n, k) holds channels 8k .. 8k + 7 of pixel (row + dy, n + dx) of the staged tile
      const int w0 = ((row + t / 3) * TP + ln + t % 3) * (PW / 2) + 4 * kg;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ts[q] + w0));
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[t][mb], b, acc[mb], 0, 0, 0);
      }
    }
    // lane (n, k) holds output channels 16 mb + 4k + j of pixel n of the row
    const int y = y0 + row;
    if (x < W && y < H) {
      float* ob = out + (size_t)n * C * plane + (size_t)y * W + x;
      const float* mb_ = mask ? mask + (size_t)n * C * plane + (size_t)y * W + x : nullptr;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int co = 16 * mb + 4 * kg + j;
          float v = acc[mb][j] + bv[mb][j];
          if (relu) v = fmaxf(v, 0.0f);
          if (mb_) v = mb_[co * plane] > 0.0f ? v : 0.0f;
          ob[co * plane] = v;
        }
    }
  }
}

// Weight gradient of a 32 -> 32 layer on the BF16 matrix cores, partial over a range of tiles: per tap t
// the GEMM dW_t[co][ci] = sum_p dout[co][p] in[ci][p + off_t] (v_mfma_f32_16x16x32_bf16), M = 16 output
// channels, N = 16 input channels, K = 32 pixels of two tile rows (8 consecutive pixels per lane).  Both
// FP32 operands are split into three BF16 parts as in conv32_mfma_kernel, and the six part products of
// order up to 2 are summed in FP32 (the dropped ones are below 2^-26 of a product).  The input tile (with
// its 1-pixel halo, rows of 24 halves) and the output-gradient tile are staged in LDS, channel-major; a
// lane's 8 pixels shifted by dx = 1, 2 come from two aligned 16-byte reads.  Wave w takes the channel
// blocks (mb, nb) = (w / 2, w % 2) for all nine taps; db[co] = sum_p dout[co][p] on the VALU, reduced in a
// fixed order.  Grid (tile groups, images); partial: [gridDim.y][gridDim.x][COUT*CIN*9 + COUT].
__global__ __launch_bounds__(256) void wgrad32_mfma_kernel(const float* __restrict__ in, const float* __restrict__ dout,
                                                           float* __restrict__ partial, int H, int W,
                                                           int tiles_per_block) {
  constexpr int C = 32, NP = C * C * 9 + C, TP = TS + 2, IW = 24;
  __shared__ __attribute__((aligned(16))) unsigned short sin_[3][C][TP][IW];
  __shared__ __attribute__((aligned(16))) unsigned short sd[3][C][TS][TS];
  __shared__ float bred[4][C];
  const int tid = threadIdx.x, lane = tid & 63, ln = lane & 15, kg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), mb = wave >> 1, nb = wave & 1;
  const int n = blockIdx.y;
  const size_t plane = (size_t)H * W;
  const int tiles_x = (W + TS - 1) / TS, tiles_y = (H + TS - 1) / TS, ntiles = tiles_x * tiles_y;
  const float* inb = in + (size_t)n * C * plane;
  const float* db = dout + (size_t)n * C * plane;
  auto split3 = [](float v, unsigned short* p, int stride) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const __bf16 h = (__bf16)v;
      p[q * stride] = __builtin_bit_cast(unsigned short, h);
      v -= (float)h;
    }
  };
  floatx4 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  float bsum[C];
#pragma unroll
  for (int k = 0; k < C; ++k) bsum[k] = 0.0f;
  for (int tt = 0; tt < tiles_per_block; ++tt) {
    const int tile = blockIdx.x * tiles_per_block + tt;
    if (tile >= ntiles) break;
    const int x0 = (tile % tiles_x) * TS, y0 = (tile / tiles_x) * TS;
    // all loads of a pass in flight before its first LDS store
    constexpr int ITEMS = C * TP * TP, HALF = (ITEMS + 511) / 512;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float v[HALF];
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        const int i = tid + 256 * (h * HALF + k);
        const int ci = i / (TP * TP), pix = i - ci * (TP * TP), r = pix / TP, c = pix - r * TP;
        const int y = y0 + r - 1, x = x0 + c - 1;
        v[k] = (i < ITEMS && y >= 0 && y < H && x >= 0 && x < W) ? inb[ci * plane + (size_t)y * W + x] : 0.0f;
      }
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        const int i = tid + 256 * (h * HALF + k);
        if (i >= ITEMS) break;
        const int ci = i / (TP * TP), pix = i - ci * (TP * TP), r = pix / TP, c = pix - r * TP;
        split3(v[k], &sin_[0][ci][r][c], C * TP * IW);
      }
    }
    {
      const int r = tid / TS, c = tid % TS, y = y0 + r, x = x0 + c;
      const bool ok = y < H && x < W;
      float v[C];
#pragma unroll
      for (int co = 0; co < C; ++co) v[co] = ok ? db[co * plane + (size_t)y * W + x] : 0.0f;
#pragma unroll
      for (int co = 0; co < C; ++co) {
        bsum[co] += v[co];
        split3(v[co], &sd[0][co][r][c], C * TS * TS);
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < TS / 2; ++s) {
      const int row = 2 * s + (kg >> 1), col = 8 * (kg & 1);
      bf16x8 a[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) a[q] = *reinterpret_cast<const bf16x8*>(&sd[q][16 * mb + ln][row][col]);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        uint4 w0[3], w1[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          w0[q] = *reinterpret_cast<const uint4*>(&sin_[q][16 * nb + ln][row + dy][col]);
          w1[q] = *reinterpret_cast<const uint4*>(&sin_[q][16 * nb + ln][row + dy][col + 8]);
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          bf16x8 b[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const unsigned u[5] = {w0[q].x, w0[q].y, w0[q].z, w0[q].w, w1[q].x};
            uint4 o;
            if (dx == 0) o = w0[q];
            else if (dx == 1)
              o = uint4{__builtin_amdgcn_alignbyte(u[1], u[0], 2), __builtin_amdgcn_alignbyte(u[2], u[1], 2),
                        __builtin_amdgcn_alignbyte(u[3], u[2], 2), __builtin_amdgcn_alignbyte(u[4], u[3], 2)};
            else o = uint4{u[1], u[2], u[3], u[4]};
            b[q] = __builtin_bit_cast(bf16x8, o);
          }
          floatx4& r = acc[3 * dy + dx];
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], r, 0, 0, 0);
          r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], r, 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* pout = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NP;
  // lane (n, k) holds dW[16 mb + 4k + j][16 nb + n][t]
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) pout[((16 * mb + 4 * kg + j) * C + 16 * nb + ln) * 9 + t] = acc[t][j];
  // db: each wave's 64 pixel sums per channel in a fixed butterfly, then the 4 waves in order
#pragma unroll
  for (int co = 0; co < C; ++co) {
    float v = bsum[co];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) bred[wave][co] = v;
  }
  __syncthreads();
  if (tid < C) pout[C * C * 9 + tid] = ((bred[0][tid] + bred[1][tid]) + bred[2][tid]) + bred[3][tid];
}

// Weight gradient of a small layer (1 -> 32 or 32 -> 1), partial over a range of tiles: the
// input tile (with its 1-pixel halo) and the output-gradient tile are staged in LDS, and each
// thread sums one or two parameters over the staged pixels in a fixed order.
// Grid: (tile groups, images); partial: [gridDim.y][gridDim.x][CO*CI*9 + CO].
template <int CI, int CO>
__global__ __launch_bounds__(256) void wgrad_small_kernel(const float* __restrict__ in, const float* __restrict__ dout,
                                                          float* __restrict__ partial, int H, int W,
                                                          int tiles_per_block) {
  constexpr int NP = CO * CI * 9 + CO, PER = (NP + 255) / 256;
  __shared__ float sin_[CI][TS + 2][TS + 2];
  __shared__ float sd[CO][TS][TS];
  const int n = blockIdx.y;
  const size_t plane = (size_t)H * W;
  const int tiles_x = (W + TS - 1) / TS, tiles_y = (H + TS - 1) / TS, ntiles = tiles_x * tiles_y;
  const float* inb = in + (size_t)n * CI * plane;
  const float* db = dout + (size_t)n * CO * plane;
  float acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0f;
  for (int tt = 0; tt < tiles_per_block; ++tt) {
    const int tile = blockIdx.x * tiles_per_block + tt;
    if (tile >= ntiles) break;
    const int x0 = (tile % tiles_x) * TS, y0 = (tile / tiles_x) * TS;
    for (int i = threadIdx.x; i < CI * (TS + 2) * (TS + 2); i += 256) {
      const int ci = i / ((TS + 2) * (TS + 2)), r = (i / (TS + 2)) % (TS + 2), c = i % (TS + 2);
      const int y = y0 + r - 1, x = x0 + c - 1;
      sin_[ci][r][c] = (y >= 0 && y < H && x >= 0 && x < W) ? inb[ci * plane + (size_t)y * W + x] : 0.0f;
    }
    for (int i = threadIdx.x; i < CO * TS * TS; i += 256) {
      const int co = i / (TS * TS), r = (i / TS) % TS, c = i % TS;
      const int y = y0 + r, x = x0 + c;
      sd[co][r][c] = (y < H && x < W) ? db[co * plane + (size_t)y * W + x] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < CO * CI * 9) {
        const int co = i / (CI * 9), ci = (i / 9) % CI, t = i % 9, dy = t / 3, dx = t % 3;
        float s = 0.0f;
        for (int r = 0; r < TS; ++r)
#pragma unroll 4
          for (int c = 0; c < TS; ++c) s = fmaf(sd[co][r][c], sin_[ci][r + dy][c + dx], s);
        acc[k] += s;
      } else if (i < NP) {
        const int co = i - CO * CI * 9;
        float s = 0.0f;
        for (int r = 0; r < TS; ++r)
          for (int c = 0; c < TS; ++c) s += sd[co][r][c];
        acc[k] += s;
      }
    }
    __syncthreads();
  }
  float* pout = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NP;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < NP) pout[i] = acc[k];
  }
}

// grad[i] = sum_b partial[b][i] in increasing b.
__global__ void reduce_partials_kernel(const float* __restrict__ partial, int nb, int np, float* __restrict__ grad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  float s = 0.0f;
  int b = 0;
  for (; b + 8 <= nb; b += 8) {   // eight loads in flight, added in order
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = partial[(size_t)(b + k) * np + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
  }
  for (; b < nb; ++b) s += partial[(size_t)b * np + i];
  grad[i] = s;
}

// a0 = log f - shift.
__global__ void input_kernel(const float* __restrict__ f, float* __restrict__ a0, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) a0[i] = logf(f[i]) - SHIFT;
}

// w0 = log f + r; u0 = e^{w0}.
__global__ void output_kernel(const float* __restrict__ f, const float* __restrict__ r, float* __restrict__ u0, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    u0[i] = expf(logf(f[i]) + r[i]);
}

// Loss (w0 - log u_t)^2 / count summed per block in double, and d loss / d r = 2 (w0 - log u_t) / count.
__global__ __launch_bounds__(256) void loss_kernel(const float* __restrict__ f, const float* __restrict__ r,
                                                   const float* __restrict__ ut, float* __restrict__ dr, size_t n,
                                                   double* __restrict__ partial) {
  __shared__ double red[4];
  const float scale = 1.0f / (float)n;
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const float d = (logf(f[i]) + r[i]) - logf(ut[i]);
    dr[i] = 2.0f * d * scale;
    s += (double)d * (double)d;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Adam on the FP32 master parameters, then the BF16 rounding used by the kernels.
__global__ void adam_kernel(float* __restrict__ master, float* __restrict__ quant, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ g, int np, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float w = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  master[i] = w;
  quant[i] = (float)(__bf16)w;
}

// From the BF16 parameters in [co][ci][t] + [co] layout: forward taps [ci][t][co] and the
// backward-data taps [co][8 - t][ci] (flipped, transposed), per layer; biases are copied.
__global__ void relayout_kernel(const float* __restrict__ quant, float* __restrict__ wfwd, float* __restrict__ wbwd,
                                float* __restrict__ bias, const int* __restrict__ offs, const int* __restrict__ woffs,
                                const int* __restrict__ boffs) {
  const int l = blockIdx.y;
  const int ci_n = CIN[l], co_n = COUT[l], nw = co_n * ci_n * 9;
  const float* q = quant + offs[l];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nw + co_n; i += gridDim.x * 256) {
    if (i < nw) {
      const int co = i / (ci_n * 9), ci = (i / 9) % ci_n, t = i % 9;
      wfwd[woffs[l] + ((size_t)ci * 9 + t) * co_n + co] = q[i];
      wbwd[woffs[l] + ((size_t)co * 9 + (8 - t)) * ci_n + ci] = q[i];
    } else {
      bias[boffs[l] + (i - nw)] = q[i];
    }
  }
}

// The A operands of conv32_mfma_kernel from taps wt[ci][t][co] (FP32 values that are BF16 numbers):
// block (t 2 + mb, layer), lane (m, k): the 8 BF16 wt[8k + i][t][16 mb + m], i = 0..7, as 4 words.
// Layers: dir 0 the forward taps, dir 1 the backward-data taps of the 32 -> 32 layers 1 .. 4.
__global__ void mfma_taps_kernel(const float* __restrict__ wfwd, const float* __restrict__ wbwd,
                                 const int* __restrict__ woffs, uint4* __restrict__ amat) {
  const int dir = blockIdx.y / (NL - 2), l = 1 + blockIdx.y % (NL - 2);
  const int t = blockIdx.x / 2, mb = blockIdx.x % 2, lane = threadIdx.x, m = lane & 15, k = lane >> 4;
  const float* w = (dir == 0 ? wfwd : wbwd) + woffs[l];
  bf16x8 a;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (__bf16)w[((8 * k + i) * 9 + t) * 32 + 16 * mb + m];
  amat[((size_t)blockIdx.y * 18 + blockIdx.x) * 64 + lane] = __builtin_bit_cast(uint4, a);
}

}  // namespace cnn

using namespace cnn;

// Error text shared with the solver API (foe_last_error).
void foe_internal_set_error(const std::string& msg);

namespace {
foe_status cfail(foe_status st, const std::string& m) {
  foe_internal_set_error(m);
  return st;
}
#define CNN_HIP_OR(expr)                                                                            \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return cfail(FOE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
}  // namespace

struct foe_cnn {
  hipStream_t stream = nullptr;
  int np = total_params();
  int offs[NL], woffs[NL], boffs[NL];
  float *master = nullptr, *quant = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  float *wfwd = nullptr, *wbwd = nullptr, *bias = nullptr;
  uint4* amat = nullptr;   // matrix-core A operands of the 32 -> 32 layers, both directions
  int *d_offs = nullptr;
  long step = 0;
  // activation workspace, grown on demand by reserve()
  size_t cap_px = 0;
  float* act[NL + 1] = {};  // act[0] input (1 ch), act[1..5] 32 ch, act[6] output (1 ch)
  float* dbuf[2] = {};      // 32-channel gradient ping-pong
  float* partial = nullptr;
  size_t partial_cap = 0;
  double* lpart = nullptr;
};

namespace {

void cnn_free(foe_cnn* c) {
  float* bufs[] = {c->master, c->quant, c->m, c->v, c->grad, c->wfwd, c->wbwd, c->bias, c->partial,
                   c->dbuf[0], c->dbuf[1]};
  for (float* b : bufs) if (b) (void)hipFree(b);
  for (float* a : c->act) if (a) (void)hipFree(a);
  if (c->d_offs) (void)hipFree(c->d_offs);
  if (c->amat) (void)hipFree(c->amat);
  if (c->lpart) (void)hipFree(c->lpart);
  delete c;
}

// Tiles per block of the weight-gradient kernels: up to 4, fewer while the grid would hold under
// 1024 blocks.
int wgrad_tiles_per_block(int n_img, int H, int W) {
  const long tiles = (long)((W + TS - 1) / TS) * ((H + TS - 1) / TS);
  return (int)std::min<long>(4, std::max<long>(1, tiles * n_img / 1024));
}

int wgrad_groups(int n_img, int H, int W) {
  const int tiles = ((W + TS - 1) / TS) * ((H + TS - 1) / TS), tpb = wgrad_tiles_per_block(n_img, H, W);
  return (tiles + tpb - 1) / tpb;
}

foe_status reserve(foe_cnn* c, int n_img, int H, int W) {
  // conv32_mfma_kernel addresses the 32 planes of one image with 32-bit byte offsets
  if ((size_t)H * W * 32 * sizeof(float) >= ((size_t)1 << 32)) return cfail(FOE_EINVAL, "image too large (H W >= 2^25)");
  const size_t px = (size_t)n_img * H * W;
  if (px > c->cap_px) {
    for (float*& a : c->act) { if (a) (void)hipFree(a); a = nullptr; }
    for (float*& d : c->dbuf) { if (d) (void)hipFree(d); d = nullptr; }
    for (int l = 0; l <= NL; ++l) {
      const int ch = l == 0 ? 1 : COUT[l - 1];
      CNN_HIP_OR(hipMalloc(&c->act[l], sizeof(float) * ch * px));
    }
    for (float*& d : c->dbuf) CNN_HIP_OR(hipMalloc(&d, sizeof(float) * 32 * px));
    c->cap_px = px;
  }
  // weight-gradient partials: (tile groups x images) blocks of the 32 -> 32 layers
  const size_t need = (size_t)n_img * wgrad_groups(n_img, H, W) * 9248;
  if (need > c->partial_cap) {
    if (c->partial) (void)hipFree(c->partial);
    c->partial = nullptr;
    CNN_HIP_OR(hipMalloc(&c->partial, sizeof(float) * need));
    c->partial_cap = need;
  }
  return FOE_OK;
}

foe_status relayout(foe_cnn* c) {
  relayout_kernel<<<dim3(37, NL), 256, 0, c->stream>>>(c->quant, c->wfwd, c->wbwd, c->bias, c->d_offs, c->d_offs + NL,
                                                       c->d_offs + 2 * NL);
  CNN_HIP_OR(hipGetLastError());
  mfma_taps_kernel<<<dim3(18, 2 * (NL - 2)), 64, 0, c->stream>>>(c->wfwd, c->wbwd, c->d_offs + NL, c->amat);
  CNN_HIP_OR(hipGetLastError());
  return FOE_OK;
}

// A operands of 32 -> 32 layer l (1 .. NL - 2), forward or backward-data.
const uint4* amat_of(const foe_cnn* c, int l, bool backward) {
  return c->amat + ((size_t)(backward ? NL - 2 : 0) + (l - 1)) * 18 * 64;
}

void launch_conv(foe_cnn* c, int l, bool backward, const float* in, float* out, const float* mask, int n, int H,
                 int W) {
  const int ntiles = ((W + TS - 1) / TS) * ((H + TS - 1) / TS) * n;
  const unsigned grid = 8u * (unsigned)((ntiles + 7) / 8);   // xcd_tile
  const float* wf = c->wfwd + c->woffs[l];
  const float* wb = c->wbwd + c->woffs[l];
  const float* b = c->bias + c->boffs[l];
  if (!backward) {
    const int relu = l < NL - 1;
    if (l == 0)
      conv3_kernel<1, 32, 1><<<grid, 256, 0, c->stream>>>(in, wf, b, out, nullptr, H, W, n, relu);
    else if (l == NL - 1)
      conv3_kernel<32, 1, 8><<<grid, 256, 0, c->stream>>>(in, wf, b, out, nullptr, H, W, n, relu);
    else
      conv32_mfma_kernel<<<grid, 256, 0, c->stream>>>(in, amat_of(c, l, false), b, out, nullptr, H, W, n, relu);
  } else {
    // d_in = conv(d_out, flipped transposed taps) * (a_in > 0); the layer's input channels are the outputs
    if (l == NL - 1)
      conv3_kernel<1, 32, 1><<<grid, 256, 0, c->stream>>>(in, wb, nullptr, out, mask, H, W, n, 0);
    else
      conv32_mfma_kernel<<<grid, 256, 0, c->stream>>>(in, amat_of(c, l, true), nullptr, out, mask, H, W, n, 0);
  }
}

// Forward pass of n images; act[NL] receives the residual r.
foe_status forward(foe_cnn* c, const float* d_f, int n, int H, int W) {
  const size_t px = (size_t)n * H * W;
  input_kernel<<<(unsigned)std::min<size_t>((px + 255) / 256, 4096), 256, 0, c->stream>>>(d_f, c->act[0], px);
  for (int l = 0; l < NL; ++l) launch_conv(c, l, false, c->act[l], c->act[l + 1], nullptr, n, H, W);
  CNN_HIP_OR(hipGetLastError());
  return FOE_OK;
}

// Loss and gradient (into c->grad) of a batch; no update.
foe_status loss_grad(foe_cnn* c, const float* d_f, const float* d_ut, int n, int H, int W, double* loss) {
  const size_t plane = (size_t)H * W, px = (size_t)n * plane;
  foe_status st = forward(c, d_f, n, H, W);
  if (st != FOE_OK) return st;
  const int lblocks = (int)std::min<size_t>((px + 255) / 256, 1024);
  float* dr = c->dbuf[0];
  loss_kernel<<<lblocks, 256, 0, c->stream>>>(d_f, c->act[NL], d_ut, dr, px, c->lpart);
  float* dcur = dr;
  float* dnext = c->dbuf[1];
  const int groups = wgrad_groups(n, H, W), tpb = wgrad_tiles_per_block(n, H, W);
  for (int l = NL - 1; l >= 0; --l) {
    const int np = layer_params(l);
    float* g = c->grad + c->offs[l];
    if (CIN[l] == 32 && COUT[l] == 32) {
      wgrad32_mfma_kernel<<<dim3(groups, n), 256, 0, c->stream>>>(c->act[l], dcur, c->partial, H, W, tpb);
      reduce_partials_kernel<<<(np + 255) / 256, 256, 0, c->stream>>>(c->partial, groups * n, np, g);
    } else if (l == 0) {
      wgrad_small_kernel<1, 32><<<dim3(groups, n), 256, 0, c->stream>>>(c->act[0], dcur, c->partial, H, W, tpb);
      reduce_partials_kernel<<<(np + 255) / 256, 256, 0, c->stream>>>(c->partial, groups * n, np, g);
    } else {
      wgrad_small_kernel<32, 1><<<dim3(groups, n), 256, 0, c->stream>>>(c->act[l], dcur, c->partial, H, W, tpb);
      reduce_partials_kernel<<<(np + 255) / 256, 256, 0, c->stream>>>(c->partial, groups * n, np, g);
    }
    if (l == 0) break;
    launch_conv(c, l, true, dcur, dnext, c->act[l], n, H, W);
    std::swap(dcur, dnext);
  }
  CNN_HIP_OR(hipGetLastError());
  if (loss) {
    std::vector<double> lp(lblocks);
    CNN_HIP_OR(hipMemcpyAsync(lp.data(), c->lpart, sizeof(double) * lblocks, hipMemcpyDeviceToHost, c->stream));
    CNN_HIP_OR(hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (double x : lp) s += x;
    *loss = s / (double)px;
  }
  return FOE_OK;
}

}  // namespace

extern "C" {

int64_t foe_cnn_num_params(void) { return total_params(); }

foe_status foe_cnn_create(const float* params_host, void* hip_stream, foe_cnn** out) {
  if (!out || !params_host) return cfail(FOE_EINVAL, "NULL argument");
  foe_cnn* c = new (std::nothrow) foe_cnn();
  if (!c) return cfail(FOE_ENOMEM, "host allocation failed");
  c->stream = (hipStream_t)hip_stream;
  int o = 0, wo = 0, bo = 0;
  for (int l = 0; l < NL; ++l) {
    c->offs[l] = o; c->woffs[l] = wo; c->boffs[l] = bo;
    o += layer_params(l); wo += COUT[l] * CIN[l] * 9; bo += COUT[l];
  }
  const size_t pb = sizeof(float) * c->np;
  bool ok = hipMalloc(&c->master, pb) == hipSuccess && hipMalloc(&c->quant, pb) == hipSuccess &&
            hipMalloc(&c->m, pb) == hipSuccess && hipMalloc(&c->v, pb) == hipSuccess &&
            hipMalloc(&c->grad, pb) == hipSuccess && hipMalloc(&c->wfwd, pb) == hipSuccess &&
            hipMalloc(&c->wbwd, pb) == hipSuccess && hipMalloc(&c->bias, pb) == hipSuccess &&
            hipMalloc(&c->d_offs, sizeof(int) * 3 * NL) == hipSuccess &&
            hipMalloc(&c->amat, sizeof(uint4) * 2 * (NL - 2) * 18 * 64) == hipSuccess &&
            hipMalloc(&c->lpart, sizeof(double) * 1024) == hipSuccess;
  if (!ok) {
    cnn_free(c);
    return cfail(FOE_ENOMEM, "device allocation failed");
  }
  std::vector<float> q(c->np);
  for (int i = 0; i < c->np; ++i) q[i] = (float)(__bf16)params_host[i];
  int offs3[3 * NL];
  for (int l = 0; l < NL; ++l) { offs3[l] = c->offs[l]; offs3[NL + l] = c->woffs[l]; offs3[2 * NL + l] = c->boffs[l]; }
  hipError_t e = hipMemcpy(c->master, params_host, pb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->quant, q.data(), pb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(c->m, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->v, 0, pb, c->stream);
  if (e == hipSuccess) e = hipMemcpy(c->d_offs, offs3, sizeof(offs3), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cnn_free(c);
    return cfail(FOE_EDEVICE, std::string("foe_cnn_create: ") + hipGetErrorString(e));
  }
  foe_status st = relayout(c);
  if (st == FOE_OK && hipStreamSynchronize(c->stream) != hipSuccess) st = cfail(FOE_EDEVICE, "relayout failed");
  if (st != FOE_OK) {
    cnn_free(c);
    return st;
  }
  *out = c;
  return FOE_OK;
}

foe_status foe_cnn_destroy(foe_cnn* c) {
  if (!c) return cfail(FOE_EINVAL, "NULL argument");
  (void)hipStreamSynchronize(c->stream);
  cnn_free(c);
  return FOE_OK;
}

foe_status foe_cnn_get_params(foe_cnn* c, float* master_host, float* bf16_host) {
  if (!c) return cfail(FOE_EINVAL, "NULL argument");
  if (master_host)
    CNN_HIP_OR(hipMemcpyAsync(master_host, c->master, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->stream));
  if (bf16_host)
    CNN_HIP_OR(hipMemcpyAsync(bf16_host, c->quant, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->stream));
  CNN_HIP_OR(hipStreamSynchronize(c->stream));
  return FOE_OK;
}

foe_status foe_cnn_infer(foe_cnn* c, const float* d_f, int32_t n, int32_t H, int32_t W, float* d_u0) {
  if (!c || !d_f || !d_u0 || n < 1 || H < 1 || W < 1) return cfail(FOE_EINVAL, "bad argument");
  const size_t px = (size_t)n * H * W;
  foe_status st = reserve(c, n, H, W);
  if (st != FOE_OK) return st;
  st = forward(c, d_f, n, H, W);
  if (st != FOE_OK) return st;
  output_kernel<<<(unsigned)std::min<size_t>((px + 255) / 256, 4096), 256, 0, c->stream>>>(d_f, c->act[NL], d_u0, px);
  CNN_HIP_OR(hipGetLastError());
  CNN_HIP_OR(hipStreamSynchronize(c->stream));
  return FOE_OK;
}

foe_status foe_cnn_loss_grad(foe_cnn* c, const float* d_f, const float* d_target_u, int32_t n, int32_t H, int32_t W,
                             double* loss, float* grad_host) {
  if (!c || !d_f || !d_target_u || n < 1 || H < 1 || W < 1) return cfail(FOE_EINVAL, "bad argument");
  foe_status st = reserve(c, n, H, W);
  if (st != FOE_OK) return st;
  st = loss_grad(c, d_f, d_target_u, n, H, W, loss);
  if (st != FOE_OK) return st;
  if (grad_host) {
    CNN_HIP_OR(hipMemcpyAsync(grad_host, c->grad, sizeof(float) * c->np, hipMemcpyDeviceToHost, c->stream));
    CNN_HIP_OR(hipStreamSynchronize(c->stream));
  }
  return FOE_OK;
}

foe_status foe_cnn_train_step(foe_cnn* c, const float* d_f, const float* d_target_u, int32_t n, int32_t H, int32_t W,
                              double lr, double* loss) {
  if (!c || !d_f || !d_target_u || n < 1 || H < 1 || W < 1 || !(lr > 0.0)) return cfail(FOE_EINVAL, "bad argument");
  foe_status st = reserve(c, n, H, W);
  if (st != FOE_OK) return st;
  st = loss_grad(c, d_f, d_target_u, n, H, W, loss);
  if (st != FOE_OK) return st;
  c->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)c->step), c2 = 1.0f - std::pow(b2, (float)c->step);
  adam_kernel<<<(c->np + 255) / 256, 256, 0, c->stream>>>(c->master, c->quant, c->m, c->v, c->grad, c->np, (float)lr, b1,
                                                         b2, 1e-8f, c1, c2);
  CNN_HIP_OR(hipGetLastError());
  st = relayout(c);
  if (st != FOE_OK) return st;
  CNN_HIP_OR(hipStreamSynchronize(c->stream));
  return FOE_OK;
}

}  // extern "C"
