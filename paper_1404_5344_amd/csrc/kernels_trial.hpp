// Fused FoE trial kernel.  The filter bank runs on one of four engines: the split-FP16 matrix-core
// engine (forward bank with FP32 operands as FP16 heads and scaled tails, adjoint on the VALU), the FP32
// matrix-core engine (forward), the BF16 engine (the split-FP16 forward, so that the energies of the line
// search keep FP32 accuracy, and the adjoint bank as a BF16 matrix-core GEMM), or the VALU direct
// convolution; the rest of the trial is the same code.
//
// One workgroup owns one TH x TW output tile and runs, entirely on chip:
//   1. the inertial step and the pointwise prox on the tile + 6-pixel halo
//      (x+ = prox_{aG}(x - a grad F(x) + b (x - x_prev)), Sec. II-C, eq. (fplusg)),
//      then u+ = e^{x+} (log models) into LDS;
//   2. per chunk of NC filters: the forward bank y_i = K_i u+ on the tile + 3 halo,
//      z_i = y_i / (1 + y_i^2) = rho'(y_i) / 2 into LDS, and theta_i rho(y_i) summed over the tile
//      (F(x+), Sec. II-A, eq. (FOEmodel));
//   3. per chunk: the adjoint bank sum_i theta_i K_i^T rho'(y_i) = sum_i K_i^T z_i with the taps
//      scaled by 2 theta_i (correlation, Sec. II-C), plus the mirror terms of the SYMMETRIC map;
//   4. the chain rule grad_w F = u .* sum_i K_i^T z_i, written as the gradient at x+
//      for the next iteration (speculative: used only if the trial is accepted),
//      and per-block partial sums {F(x+), G(x+), <grad F(x), d>, |d|^2, |x - x_prev|^2}.
// In EVAL mode stage 1 is the identity (x+ = x_in): F, G and grad F at x_in.
#pragma once
#include <type_traits>

#include "device_math.hpp"

namespace foe {

enum FusedMode { MODE_TRIAL = 0, MODE_EVAL = 1 };
// Engines: FWD_MFMA_BF16 takes the forward of FWD_MFMA_F16X and the BF16 matrix-core adjoint (ZStrips).
enum ForwardEngine { FWD_VALU = 0, FWD_MFMA_F32 = 1, FWD_MFMA_BF16 = 2, FWD_MFMA_F16X = 3 };
// Fusion of the gradient: the whole trial in one kernel (FUSED), or split in two launches that
// exchange the 48 z planes through HBM: FWD_HALF runs stages 1-2 (step, prox, forward bank,
// energies) and stores z_i on the tile, ADJ_HALF loads z_i on the tile + 3 halo and runs stage 3
// and the chain rule.
enum Fusion { FUSED = 0, FWD_HALF = 1, ADJ_HALF = 2 };
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct FusedArgs {
  Problem pb;
  const TileDesc* tiles;                // [gridDim.x]
  const ImageDesc* images;
  const float* f;                       // packed planes of all images
  float* xr0; float* xr1; float* xr2;   // x ring (TRIAL), packed
  float* gr0; float* gr1;               // gradient ring (TRIAL), packed
  const float* x_in;                    // EVAL input, packed
  float* g_out;                         // EVAL output, packed
  DevState* st;                         // per-image states (read)
  double* partials;                     // [gridDim.x][PART_COLS] (written)
  // decide_prev: before its own trial every workgroup reduces part_in (the previous trial's partials) over
  // its image's tiles and applies the line-search decision to a copy of st; the image's first workgroup
  // stores the decided state (pending = 1 unless done) to st_out and the accepted stats row.
  int decide_prev;
  DevState* st_out;
  const double* part_in;
  double* stats;                        // [images][stats_rows][STAT_COLS]
  int stats_rows;
  const float* kf;                      // forward taps, flipped and chunk-transposed:
                                        //   kf[(c * KK + a * 7 + b) * NC + j] = k_{c*NC+j}[6-a][6-b]
  const float* ka;                      // adjoint taps: ka[i][a][b] = 2 theta_i k_i[a][b]
  const unsigned* kf16;                 // split-FP16 forward operands: per chunk, F16_OPS words in the
                                        //   lane order of the split engine (ForwardOps<FWD_MFMA_F16X>)
  const unsigned* kb16;                 // BF16 adjoint operands (matrix-core adjoint): KB16_W words per
                                        //   filter (ZStrips)
  const float* theta;
  float* zbuf;                          // unfused z planes: zbuf[i * zstride + off + y * W + x]
  long long zstride;
  int mode;
};

// Block-wide deterministic sum of NV doubles per thread -> partials[blockIdx.x][0..NV).
template <int NT, int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_f64(v[k]);
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w * NV + threadIdx.x];
    out[(size_t)blockIdx.x * PART_COLS + threadIdx.x] = s;
  }
}

// z lines of the fold: Z_r[s] = z at line r, position s along the line, from FP32 planes (B16 = false) or
// from the BF16 engine's strips (B16 = true).
template <int ZS, int ZL, bool B16 = false>
struct ZLines {
  const void* p;
  __device__ __forceinline__ float operator()(int r, int s) const {
    if constexpr (B16)
      return (float)static_cast<const __bf16*>(p)[r * ZL + s * ZS];
    else
      return static_cast<const float*>(p)[r * ZL + s * ZS];
  }
};

// The mirror terms of FB consecutive positions along an edge for one filter: v_i(d) = sum_{r <= 2 - d}
// <K_{d+r}, Z_r[i .. i + 6]> with Z_r[s] the z line at distance r from the edge (s = 0 .. FB + 5) and K_m the
// tap line 4 + m (low edge) or 2 - m (high edge), added to out[(i R + d) NC] (each partial has one writer per
// chunk).
template <int FB, int NC>
__device__ __forceinline__ void fold_sums(const float (&Z)[R][FB + KS - 1], const float (&K)[R][KS], float* out) {
#pragma unroll
  for (int i = 0; i < FB; ++i) {
    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      v0 = fmaf(K[0][t], Z[0][i + t], v0);
      v0 = fmaf(K[1][t], Z[1][i + t], v0);
      v0 = fmaf(K[2][t], Z[2][i + t], v0);
      v1 = fmaf(K[1][t], Z[0][i + t], v1);
      v1 = fmaf(K[2][t], Z[1][i + t], v1);
      v2 = fmaf(K[2][t], Z[0][i + t], v2);
    }
    out[(i * R + 0) * NC] += v0;
    out[(i * R + 1) * NC] += v1;
    out[(i * R + 2) * NC] += v2;
  }
}

// fold_sums with Z_r[s] = zl(r, s) and K_m[t] = kb[m KL + t KT], read one value at a time.
template <int FB, int NC, int KT, int KL, class ZL>
__device__ __forceinline__ void fold_block(ZL zl, const float* kb, float* out) {
  float Z[R][FB + KS - 1], K[R][KS];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int s = 0; s < FB + KS - 1; ++s) Z[r][s] = zl(r, s);
#pragma unroll
    for (int t = 0; t < KS; ++t) K[r][t] = kb[r * KL + t * KT];
  }
  fold_sums<FB, NC>(Z, K, out);
}

// fold_sums on a y edge of the FP32 planes.  zl: the edge line (plane row) at column p0, from an 8-byte boundary
// (even plane and row strides, even p0); the lines run away from the edge by zs = +ZW (low edge) or -ZW (high).
// ka_j: the filter's adjoint taps from a 16-byte boundary; the tap lines 4..6 (low) or 2..0 (high) are the 21
// consecutive taps 28..48 or 0..20.  Pairs and quads of consecutive values are read together.
template <int FB, int NC, bool LO>
__device__ __forceinline__ void fold_block_y(const float* zl, int zs, const float* ka_j, float* out) {
  static_assert((FB + KS - 1) % 2 == 0, "the z lines read as pairs");
  float Z[R][FB + KS - 1], K[R][KS], kb[24];
  const float4* k4 = reinterpret_cast<const float4*>(ka_j + (LO ? (R + 1) * KS : 0));
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const float4 v = k4[q];
    kb[4 * q] = v.x; kb[4 * q + 1] = v.y; kb[4 * q + 2] = v.z; kb[4 * q + 3] = v.w;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int t = 0; t < KS; ++t) K[r][t] = kb[(LO ? r : R - 1 - r) * KS + t];
    const float* zr = zl + r * zs;
#pragma unroll
    for (int s = 0; s < FB + KS - 1; s += 2) {
      const float2 v = *reinterpret_cast<const float2*>(zr + s);
      Z[r][s] = v.x;
      Z[r][s + 1] = v.y;
    }
  }
  fold_sums<FB, NC>(Z, K, out);
}

// fold_sums on an x edge of the FP32 planes.  zl: row p0 of the plane (an even float offset), zcol: the plane
// column of the edge line (R on the low edge), zw: the row stride (even); the lines are the columns zcol, zcol +
// 1, zcol + 2 (low) or zcol, zcol - 1, zcol - 2 (high), each three taken as one pair and one single value.  The
// tap lines are the columns 4..6 (low) or 2..0 (high) of every tap row of ka_j (16-byte aligned).
template <int FB, int NC, bool LO>
__device__ __forceinline__ void fold_block_x(const float* zl, int zw, int zcol, const float* ka_j, float* out) {
  float Z[R][FB + KS - 1], K[R][KS];
#pragma unroll
  for (int t = 0; t < KS; ++t) {
    // low: taps 7t + 4 + r; high: taps 7t + 2 - r.  b: the lowest of the three (its parity is known once t is)
    const int b = KS * t + (LO ? R + 1 : 0);
    if (b % 2 == 0) {
      const float2 v = *reinterpret_cast<const float2*>(ka_j + b);
      const float w = ka_j[b + 2];
      if (LO) { K[0][t] = v.x; K[1][t] = v.y; K[2][t] = w; }
      else { K[2][t] = v.x; K[1][t] = v.y; K[0][t] = w; }
    } else {
      const float w = ka_j[b];
      const float2 v = *reinterpret_cast<const float2*>(ka_j + b + 1);
      if (LO) { K[0][t] = w; K[1][t] = v.x; K[2][t] = v.y; }
      else { K[2][t] = w; K[1][t] = v.x; K[0][t] = v.y; }
    }
  }
  const int c0 = LO ? zcol : zcol - (R - 1);   // the lowest of the three columns
  if (c0 % 2 == 0) {
#pragma unroll
    for (int s = 0; s < FB + KS - 1; ++s) {
      const float2 v = *reinterpret_cast<const float2*>(zl + s * zw + c0);
      const float w = zl[s * zw + c0 + 2];
      if (LO) { Z[0][s] = v.x; Z[1][s] = v.y; Z[2][s] = w; }
      else { Z[2][s] = v.x; Z[1][s] = v.y; Z[0][s] = w; }
    }
  } else {
#pragma unroll
    for (int s = 0; s < FB + KS - 1; ++s) {
      const float w = zl[s * zw + c0];
      const float2 v = *reinterpret_cast<const float2*>(zl + s * zw + c0 + 1);
      if (LO) { Z[0][s] = w; Z[1][s] = v.x; Z[2][s] = v.y; }
      else { Z[2][s] = w; Z[1][s] = v.x; Z[0][s] = v.y; }
    }
  }
  fold_sums<FB, NC>(Z, K, out);
}

// Operands of the matrix-core forward bank that stay in registers for one chunk of 16 filters.
//   FP32 engine: taps 0..47 in twelve steps of v_mfma_f32_16x16x4f32 (lane (m, k): A = filter m at
//   tap 4s + k, B = u6 at that tap of position m); the VALU adds tap 48.
//   Split-FP16 engine: the 7 x 7 taps laid out as 8 x 8 (tap row, tap column; row 7 and column 7
//   zero) in two steps of v_mfma_f32_16x16x32_f16: in step s lane (m, k) holds tap row 4s + k,
//   columns 0..7, of filter m (A) and of position m (B).  Every FP32 operand v is split into two FP16
//   numbers, v = hi + lo / 4096 with hi = fp16(v), lo = fp16(4096 (v - hi)), which keeps about 22
//   significant bits of v; y = hi.hi + (lo.hi + hi.lo) / 4096, where every product of two FP16
//   numbers is exact in FP32 and only the lo.lo term (2^-22 of the product) is dropped.  u is split
//   after scaling by the tile's power of two 2^-E (largest |u| of the tile in [2^13, 2^14)), so that
//   no u of any range overflows FP16; y is scaled back by 2^E.
constexpr int F16_OPS = 64 * 16;   // words of split-FP16 tap operands per chunk: 16 per lane
template <int FWD> struct ForwardOps;
template <> struct ForwardOps<FWD_MFMA_F32> {
  float a[KK / 4];
  int toff[KK / 4];
  float4 klast;
};
template <> struct ForwardOps<FWD_MFMA_F16X> {
  half8 hi[2], lo[2];   // A operands of the two steps (FP16 heads, 4096-scaled tails)
  float sc, sclo;       // 2^E and 2^(E - 12)
};
template <> struct ForwardOps<FWD_MFMA_BF16> : ForwardOps<FWD_MFMA_F16X> {};

// Row stride of the z planes (the tile + 3 halo, TW + 6 wide): the split engine pads it to a multiple of 8
// floats, so that the adjoint's 10-wide window rows load as two 16-byte reads and a pair, and the
// 2 x 8 position patches of its forward store z into distinct LDS banks.
constexpr bool split_forward(int fwd) { return fwd == FWD_MFMA_F16X || fwd == FWD_MFMA_BF16; }
constexpr int z_row_stride(int tw, int fwd) { return split_forward(fwd) ? (tw + 2 * R + 7) / 8 * 8 : tw + 2 * R; }
// Stride of the z planes: with padded rows the plane is padded too, to 4 (mod 64) floats, so that lanes
// that read the same position of 16 different planes (the fold) fall in 16 different banks.
constexpr int z_plane_stride(int tw, int th, int fwd) {
  return split_forward(fwd) ? (th + 2 * R) * z_row_stride(tw, fwd) + ((4 - (th + 2 * R) * z_row_stride(tw, fwd) % 64) % 64 + 64) % 64
                              : (th + 2 * R) * (tw + 2 * R);
}

// LDS planes of the split-FP16 engine: u6 / 2^E as FP16 heads and tails, row by row ([head row][tail
// row], COLS halves each), in two copies: copy 0 holds column c at c, copy 1 holds column c + 1 at c,
// so that the 8 consecutive columns of a B operand start on a 4-byte boundary in one of them.  One
// padding row and the padding columns hold zeros: they meet the zero taps of row 7 and column 7.
// Copy 1 starts at a word offset of 23 (mod 64): with the 2 x 8 position patches of the forward, the
// B loads of a wave then fall in distinct banks (64 banks of 4 bytes) for either column parity.
template <int TW, int TH>
struct SplitPlanes {
  static constexpr int W6 = TW + 4 * R, H6 = TH + 4 * R;
  static constexpr int COLS = W6 + 2;            // halves per head / tail row (even)
  static constexpr int ROWS = H6 + 1;
  static constexpr int ROW_W = COLS;             // words per plane row (head + tail)
  static constexpr int COPY_W = ROWS * ROW_W;    // words per copy
  static constexpr int COPY1 = COPY_W + ((23 - COPY_W % 64) % 64 + 64) % 64;   // word offset of copy 1
  static constexpr int WORDS = COPY1 + COPY_W;
  static constexpr int TAIL_W = COLS / 2;        // word offset of the tail row
};

// Writes v (= u6[r][c] / 2^E) as its FP16 head and 4096-scaled FP16 tail into both plane copies.
template <int TW, int TH>
__device__ __forceinline__ void split_store(unsigned* u16w, int r, int c, float v) {
  using SP = SplitPlanes<TW, TH>;
  const _Float16 hi = (_Float16)v;
  const _Float16 lo = (_Float16)((v - (float)hi) * 4096.0f);
  _Float16* q = reinterpret_cast<_Float16*>(u16w) + r * 2 * SP::ROW_W + c;
  q[0] = hi;
  q[SP::COLS] = lo;
  if (c > 0) {   // copy 1 holds column c at c - 1
    q[2 * SP::COPY1 - 1] = hi;
    q[2 * SP::COPY1 - 1 + SP::COLS] = lo;
  }
}

// z planes of the BF16 engine's matrix-core adjoint.  The adjoint of one filter on a 16 x 16 output block
// (rows r0 .. r0 + 15, columns 16 s .. 16 s + 15 of the tile) is a Toeplitz GEMM on
// v_mfma_f32_16x16x32_bf16:
//   g(r0 + m, 16 s + n) = sum_{a, b} ka[a][b] z3(r0 + m + a, 16 s + n + b) = sum_k A[m][k] B[k][n],
// with the z window of the block kept as a strip of W = 22 columns (16 + 6) per row, flattened row-major:
// A[m][k] = strip(r0 + m)[k] for k = 22 a + c (k < 160: the flattening runs on into the next rows, which meet
// zero taps), and B[k][n] = T[k - n], T[22 a + b] = ka[a][b] for b < 7, zero for b in [7, 22) and outside
// [0, 154).  A tile of TW = 32 columns takes two strips (z3 columns 0 .. 21 and 16 .. 37).  Operands are
// BF16 (z in [-1/2, 1/2] and the taps each rounded once), products and sums FP32.  Layout per filter j:
// strips 0, 1 of STRIP_H halves each; a padding of 8 halves after the last filter holds zeros (the last rows'
// k >= 154 reads).
template <int TW, int TH>
struct ZStrips {
  static constexpr int H3 = TH + 2 * R, W3 = TW + 2 * R;
  static constexpr int W = 22;                       // strip columns: 16 outputs + 6
  static constexpr int NS = TW / 16;                 // strips per tile row
  static constexpr int STRIP_H = H3 * W;             // halves per strip
  static constexpr int FILTER_H = NS * STRIP_H;      // halves per filter
  static constexpr int KSTEPS = (KS * W + 31) / 32;  // 32-wide K steps: 5
  static constexpr int NB = (TH / 16) * NS;          // 16 x 16 output blocks per tile
  static_assert(TW == 32 && TH % 16 == 0 && W3 == 16 * (NS - 1) + W, "two strips cover the tile + 3 halo");
  static_assert(KSTEPS * 32 - KS * W <= W, "the flattened K range ends inside the next row");
};
// BF16 adjoint tap operands in global memory, per filter: T padded by 16 zeros in front and zeros behind, in
// two copies (copy 1 shifted by one half), so that the 8 consecutive values T[32 s + 8 kb - n .. + 7] of lane
// (n, kb) start on a 4-byte boundary in copy n & 1.  Word w of copy c of filter i: kb16[i * KB16_W + c *
// KB16_COPY + w].
constexpr int KB16_COPY = 88;               // 176 halves: T[-16 .. 159]
constexpr int KB16_W = 2 * KB16_COPY;

// The live and own bits (bits 2i and 2i + 1) of the passes i of lane m of wave g0 in the split engine's
// 2 x 8 patch groups: the same in every chunk, so they are formed once per launch.  Every pass is tested
// with its own row and column in vector registers (g0 is the wave index taken per lane): a few VALU
// instructions per pass, where scalar loop code would queue the 16 waves of the workgroup on the one
// scalar unit of the CU.  Bits of passes past the last group are never read.
template <int TW, int TH, int GS>
__device__ __forceinline__ unsigned patch_masks(int g0, int lm, int y0, int x0, int H, int W, bool periodic) {
  constexpr int W3 = TW + 2 * R, H3 = TH + 2 * R, NCB = (W3 + 7) / 8, NG = (H3 / 2) * NCB;
  constexpr int NPASS = (NG + GS - 1) / GS;
  static_assert(2 * NPASS <= 32 && NCB <= 32, "two bits per pass");
  const int dy = lm >> 3, dx = lm & 7;
  unsigned m = 0u;
#pragma unroll
  for (int i = 0; i < NPASS; ++i) {
    const int g = g0 + i * GS;
    const int rp = g / NCB, cb = g - rp * NCB;
    const int rr = 2 * rp + dy, cc = 8 * cb + dx;
    const bool inimg = (unsigned)(y0 - R + rr) < (unsigned)H && (unsigned)(x0 - R + cc) < (unsigned)W;
    const bool own = inimg && (unsigned)(rr - R) < (unsigned)TH && (unsigned)(cc - R) < (unsigned)TW;
    m |= (unsigned)(inimg || periodic) << (2 * i);
    m |= (unsigned)own << (2 * i + 1);
  }
  return m;
}

// One chunk of the matrix-core forward bank on the R3 region of a TW x TH tile: the position groups
// g0, g0 + GS, ... of 16 positions each (FP32 engine: 16 consecutive positions; split engine: 2 x 8
// patches), with the operands of ForwardOps<FWD>; lane (m, k) then holds y for position m of the
// group, filters 4k .. 4k + 3, and stores z = y / (1 + y^2) into the z planes.  Returns this thread's
// sum of theta ln(1 + y^2) over its own (tile, in-image) positions.  ALL_IN: every R3 position lies in
// the image, so that no z needs masking and every tile position is an own one.  FUSION == FWD_HALF
// also stores z of the own positions to HBM (zb = plane of the chunk's first filter at the image,
// zstride apart).  UNIT: the tile's u was not scaled (2^E = 1).  Lanes without a position of their own
// in a group repeat one that another lane holds, from the same operands: they store the same bits
// again, and the position is a halo one, so it adds no energy.
template <int TW, int TH, int NC, int GS, int FUSION, bool ALL_IN, int FWD, bool UNIT = false>
__device__ __forceinline__ float mfma_forward_chunk(const float* u6, const unsigned* u16, float* zp,
                                                    const ForwardOps<FWD>& ops, const float (&thl)[4], int g0, int lm,
                                                    int lk, int y0, int x0, int H, int W, bool periodic, float* zb,
                                                    long long zstride, int nlive, unsigned pmask) {
  using SP = SplitPlanes<TW, TH>;
  constexpr int W6 = TW + 4 * R, W3 = TW + 2 * R, H3 = TH + 2 * R;
  constexpr int ZW = z_row_stride(TW, FWD), PLANE = z_plane_stride(TW, TH, FWD), PLANE3 = H3 * W3;
  constexpr int TLAST = (KS - 1) * W6 + (KS - 1);
  // the fused BF16 engine keeps z as BF16 strips for its matrix-core adjoint (ZStrips)
  constexpr bool ZSPLIT = FWD == FWD_MFMA_BF16 && FUSION == FUSED;
  float ef = 0.0f;
  // one group: this lane's position (rr, cc) of the R3 region; live: z is kept (in the image, or periodic);
  // own: a tile position in the image, whose energy counts.  zq: the position in plane 0 (FP32 planes);
  // zh0 / zh1: the position in strip 0 / 1 of filter 0, stored when s0 / s1 (ZSPLIT)
  auto group = [&](int rr, int cc, const unsigned* b, float* zq, __bf16* zh0, __bf16* zh1, bool s0, bool s1,
                   bool live, bool own) {
    floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (FWD == FWD_MFMA_F32) {
      const int pbase = rr * W6 + cc;
#pragma unroll
      for (int s = 0; s < KK / 4; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ops.a[s], u6[pbase + ops.toff[s]], acc, 0, 0, 0);
      const float ulast = u6[pbase + TLAST];
      acc[0] = fmaf(ops.klast.x, ulast, acc[0]);
      acc[1] = fmaf(ops.klast.y, ulast, acc[1]);
      acc[2] = fmaf(ops.klast.z, ulast, acc[2]);
      acc[3] = fmaf(ops.klast.w, ulast, acc[3]);
    } else {
      // b: window row rr + lk, columns cc .. cc + 7, in the copy where they are aligned (+ 4 rows in
      // step 1)
      floatx4 hh = {0.0f, 0.0f, 0.0f, 0.0f}, cr = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int o = s * 4 * SP::ROW_W, ot = o + SP::TAIL_W;
        const u32x4 wh = {b[o], b[o + 1], b[o + 2], b[o + 3]};
        const u32x4 wt = {b[ot], b[ot + 1], b[ot + 2], b[ot + 3]};
        const half8 bh = __builtin_bit_cast(half8, wh), bt = __builtin_bit_cast(half8, wt);
        cr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ops.lo[s], bh, cr, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ops.hi[s], bt, cr, 0, 0, 0);
        hh = __builtin_amdgcn_mfma_f32_16x16x32_f16(ops.hi[s], bh, hh, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = UNIT ? fmaf(cr[j], 1.0f / 4096.0f, hh[j]) : fmaf(cr[j], ops.sclo, hh[j] * ops.sc);
    }
    const int gy = y0 - R + rr, gx = x0 - R + cc;
    float e = 0.0f, zv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float yv = acc[j];
      const float den = fmaf(yv, yv, 1.0f);
      const float z = yv * fast_rcp(den);
      zv[j] = live ? z : 0.0f;
      if constexpr (!ZSPLIT) zq[(4 * lk + j) * PLANE] = zv[j];   // zq: this position in plane 0
      if (FUSION == FWD_HALF && own && 4 * lk + j < nlive) zb[(4 * lk + j) * zstride + (long long)gy * W + gx] = z;
      e = fmaf(thl[j], __builtin_amdgcn_logf(den), e);   // theta ln 2 * log2(1 + y^2)
    }
    if constexpr (ZSPLIT) {
      // BF16 pairs of two neighbouring columns: lanes 2i and 2i + 1 of a row hold columns cc and cc + 1 of the
      // same four filters; they swap two values (DPP quad_perm 1, 0, 3, 2), then the even lane stores filters
      // 4k, 4k + 1 and the odd lane filters 4k + 2, 4k + 3 as one word each (low half = the even column)
      const bool odd = lm & 1;   // the lane's column parity (cc = 8 cb + (lm & 7))
      const float ra = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(odd ? zv[0] : zv[2]), 0xb1, 0xf, 0xf, false));
      const float rb = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(odd ? zv[1] : zv[3]), 0xb1, 0xf, 0xf, false));
      auto pack = [](float lo, float hi) {
        return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)lo) |
               ((unsigned)__builtin_bit_cast(unsigned short, (__bf16)hi) << 16);
      };
      const unsigned wa = odd ? pack(ra, zv[2]) : pack(zv[0], ra);
      const unsigned wb = odd ? pack(rb, zv[3]) : pack(zv[1], rb);
      const int fo = (4 * lk + (odd ? 2 : 0)) * ZStrips<TW, TH>::FILTER_H - (odd ? 1 : 0);
      constexpr int FW = ZStrips<TW, TH>::FILTER_H / 2;
      if (s0) {
        unsigned* w = reinterpret_cast<unsigned*>(zh0 + fo);
        w[0] = wa;
        w[FW] = wb;
      }
      if (s1) {
        unsigned* w = reinterpret_cast<unsigned*>(zh1 + fo);
        w[0] = wa;
        w[FW] = wb;
      }
    }
    ef += own ? e : 0.0f;
  };
  if constexpr (FWD == FWD_MFMA_F32) {
    // groups of 16 consecutive positions; lanes past the plane in the last group take position 0
    constexpr int NGROUP = (PLANE3 + 15) / 16, NFULL = PLANE3 / 16;
    constexpr int STEP = GS * 16, DR = STEP / W3, DC = STEP % W3;   // position advance per pass
    int p = g0 * 16 + lm, r = p / W3, c = p - r * W3;
    auto masks = [&](int rr, int cc, bool& live, bool& own) {
      bool inimg = true;
      if constexpr (!ALL_IN) inimg = (unsigned)(y0 - R + rr) < (unsigned)H && (unsigned)(x0 - R + cc) < (unsigned)W;
      live = ALL_IN || inimg || periodic;
      own = inimg && (unsigned)(rr - R) < (unsigned)TH && (unsigned)(cc - R) < (unsigned)TW;
    };
    int g = g0;
#pragma unroll 1
    for (; g < NFULL; g += GS) {
      bool live, own;
      masks(r, c, live, own);
      group(r, c, u16, zp + r * ZW + c, nullptr, nullptr, false, false, live, own);
      p += STEP;
      c += DC;
      r += DR;
      if (c >= W3) {
        c -= W3;
        r += 1;
      }
    }
    if (NFULL < NGROUP && g < NGROUP) {
      const int rr = p < PLANE3 ? r : 0, cc = p < PLANE3 ? c : 0;
      bool live, own;
      masks(rr, cc, live, own);
      group(rr, cc, u16, zp + rr * ZW + cc, nullptr, nullptr, false, false, live, own);
    }
  } else {
    // groups of 2 x 8 positions (lane m: row m / 8, column m % 8 of the patch), patch rows of NCB
    // patches.  The last patch of a row reaches past the region to column 8 NCB - 1: those positions lie
    // in the padding columns of the z rows (never read), their windows in the zero padding of the u
    // planes, and they are never own ones.  pmask holds the live and own bits of this lane's passes
    // (patch_masks).  A pass advances NCB-patch rows and patches by constants, so the B address b and
    // the z address zq advance by one of two constants (the wrap is the same for the whole wave).
    constexpr int NCB = (W3 + 7) / 8, NG = (H3 / 2) * NCB;
    static_assert(H3 % 2 == 0, "patches of two rows");
    static_assert(8 * NCB <= ZW && 8 * NCB + 6 <= SP::COLS, "the last patch stays inside the padded rows");
    constexpr int DR = 2 * (GS / NCB), DC = 8 * (GS % NCB);          // per pass, and + 2 / - 8 NCB on a wrap
    constexpr int DBW = DR * SP::ROW_W + DC / 2, DBW_WRAP = (DR + 2) * SP::ROW_W + (DC - 8 * NCB) / 2;
    constexpr int DZO = DR * ZW + DC, DZO_WRAP = (DR + 2) * ZW + DC - 8 * NCB;
    const int dy = lm >> 3, dx = lm & 7;
    int rp = g0 / NCB, cb = g0 - (g0 / NCB) * NCB;
    int rr = 2 * rp + dy, cc = cb * 8 + dx;
    const unsigned* b = u16 + (cc & 1) * SP::COPY1 + (rr + lk) * SP::ROW_W + (cc >> 1);
    float* zq = zp + rr * ZW + cc;
    // ZSPLIT: strip 0 takes the columns < 22, strip 1 the columns 16 .. W3 - 1 (never the padding columns)
    constexpr int SW = 22, SH = ZSPLIT ? ZStrips<ZSPLIT ? TW : 32, ZSPLIT ? TH : 16>::STRIP_H : 0;
    constexpr int DZH = DR * SW + DC, DZH_WRAP = (DR + 2) * SW + DC - 8 * NCB;
    __bf16* zh0 = reinterpret_cast<__bf16*>(zp) + rr * SW + cc;
    __bf16* zh1 = zh0 + SH - 16;
    unsigned m = pmask;
#pragma unroll 1
    for (int g = g0; g < NG; g += GS) {
      group(rr, cc, b, zq, zh0, zh1, cc < SW, cc >= 16 && cc < W3, ALL_IN || (m & 1u), (m & 2u) != 0u);
      m >>= 2;
      cb += GS % NCB;
      const bool wrap = cb >= NCB;
      if (wrap) cb -= NCB;
      rr += wrap ? DR + 2 : DR;
      cc += wrap ? DC - 8 * NCB : DC;
      b += wrap ? DBW_WRAP : DBW;
      if constexpr (ZSPLIT) {
        zh0 += wrap ? DZH_WRAP : DZH;
        zh1 += wrap ? DZH_WRAP : DZH;
      } else {
        zq += wrap ? DZO_WRAP : DZO;
      }
    }
  }
  return ef;
}

// Mirror terms of the SYMMETRIC boundary map (half-sample reflection, so x(-1-i) = x(i)).  The
// adjoint on the extended domain gives every extended sample q (within 3 of the image, off it) the
// value v(q) = sum_{a,b} k[a][b] z(q_y - 3 + a, q_x - 3 + b), and the gradient at the pixel p that q
// mirrors to receives v(q).  z vanishes off the image, so only the window lines inside the image
// count: a sample d = 0, 1, 2 lines outside an edge sees the 3 - d z lines nearest that edge through
// the tap lines 4 + d .. 6 (low edge) or 2 - d .. 0 (high edge).  With Z_r the z line at distance r
// from the edge and K_m the tap line 4 + m (low) or 2 - m (high), both taken along the edge,
//   v(d) = sum_{r=0}^{2-d} <K_{d+r}, Z_r>   (7 products per line pair).
// One fold item is one filter and FB consecutive positions along an edge (fold_block): it forms v(0),
// v(1), v(2) of each.  Items of the y edges run over the TW columns of the tile, items of the x edges
// over its TH rows; one more item per filter and corner row takes the extended rows -1-i (target row
// i) and H+i (target row H-1-i) of an x edge whose target row lies in the tile: a corner sample then
// is an x-edge position whose window rows off the image read zeros.
// Layout slots (partials fpart[(slot * 3 + d) * NC + j] in the epilogue):
//   [0, TW) y-low, [TW, 2TW) y-high, then per x edge TH + 6 slots: the tile rows, the 3 low-corner
//   rows (i = 0..2), the 3 high-corner rows (i = 0..2).

// Tile configuration: TW x TH output tile, NC filters per LDS chunk, NT threads, adjoint
// register blocks of BR x BC outputs per thread (NT / ((TH/BR) (TW/BC)) filter groups).
//
// LDS layout: u6 holds u+ on the tile + 6 halo.  Each z plane holds z_j = theta_j rho'(y_j) on
// the tile + 3 halo (R3, row stride ZW), zero off the image except under the PERIODIC map; every
// position of the planes is written in every chunk.  fpart holds the fold partials of the
// SYMMETRIC map on tiles within 3 of the image border, accumulated over the chunks.
template <int TW, int TH, int NC, int NT, int BR, int BC, int FWD, int UNF = FUSED>
__global__ __launch_bounds__(NT) void foe_trial_kernel(FusedArgs a) {
  constexpr int W6 = TW + 4 * R, H6 = TH + 4 * R;
  constexpr int W3 = TW + 2 * R, H3 = TH + 2 * R;
  constexpr int PLANE3 = H3 * W3;                 // positions of the tile + 3 halo
  constexpr int ZW = z_row_stride(TW, FWD);       // z plane row stride
  constexpr int PLANE = z_plane_stride(TW, TH, FWD);   // one z plane: the tile + 3 halo, row stride ZW
  constexpr int PPT = (PLANE3 + NT - 1) / NT;     // forward positions per thread
  constexpr int GT = (TH / BR) * (TW / BC);       // threads per adjoint group
  constexpr int NG = NT / GT;                     // filter groups
  constexpr int FPG = NC / NG;                    // filters per group per chunk
  constexpr int WR = BR + KS - 1, WC = BC + KS - 1;
  constexpr int NPX = TH + 6;                     // layout slots per x edge
  constexpr int NSLOT = 2 * TW + 2 * NPX;          // fold layout slots
  static_assert(NT % GT == 0 && NC % NG == 0 && GT % 64 == 0 && TH % BR == 0 && TW % BC == 0, "bad tiling");
  static_assert(BC % 2 == 0 && ZW % 2 == 0 && PLANE % 2 == 0, "adjoint reads float2 pairs");
  constexpr bool WIN4 = ZW % 4 == 0 && BC % 4 == 0 && PLANE % 4 == 0;   // window rows start on 16 bytes
  static_assert(NC % 8 == 0, "forward passes take 8 filters");

  static_assert((NC & (NC - 1)) == 0 && TH >= R && TW >= R, "fold items: NC a power of two, tiles >= 3");
  static_assert(FWD == FWD_VALU || NC == 16, "the MFMA forwards take one 16-filter block per chunk");
  static_assert(KK % 4 == 1, "the FP32 matrix-core forward takes taps 0 .. KK - 2 in steps of 4");
  constexpr int NGROUP = (PLANE3 + 15) / 16;      // MFMA forward: groups of 16 consecutive positions

  constexpr bool SPLIT = split_forward(FWD);   // the split-FP16 forward
  // the BF16 engine's fused kernel and adjoint half: z as BF16 strips, the adjoint bank on the matrix cores
  // (ZStrips)
  constexpr bool ZSPLIT = FWD == FWD_MFMA_BF16 && (UNF == FUSED || UNF == ADJ_HALF);
  using ZS = ZStrips<ZSPLIT ? TW : 32, ZSPLIT ? TH : 16>;   // only the BF16 engine's strips are ever used
  constexpr int ZS_WORDS = (NC * ZS::FILTER_H + 8) / 2;   // strips of the chunk + the zero padding
  constexpr int ZP_FLOATS = ZSPLIT ? (ZS_WORDS > NG * TH * TW ? ZS_WORDS : NG * TH * TW) : NC * PLANE;
  static_assert(NG * TH * TW <= ZP_FLOATS, "epilogue does not fit in the z buffer");
  static_assert(!ZSPLIT || NT / 64 == NC, "the matrix-core adjoint takes one filter of the chunk per wave");
  __shared__ float u6[H6 * W6];
  __shared__ __attribute__((aligned(16))) float zp[ZP_FLOATS];
  __shared__ float fpart[NSLOT * R * NC];  // fold partials [slot][d][filter of the chunk], over chunks
  __shared__ double red[(NT / 64) * 5];
  // taps of the current chunk, read by broadcast LDS loads so that the FMAs take them from VGPRs
  // (a VALU FMA with an SGPR operand issues at half rate on gfx950)
  constexpr int KAP = 52;                                   // padded adjoint tap stride (16 B rows)
  constexpr int KF_N = SPLIT ? F16_OPS : KK * NC;           // forward tap words per chunk
  __shared__ __attribute__((aligned(16))) float kf_s[KF_N];      // [t][j], or the split operands by lane
  __shared__ __attribute__((aligned(16))) float ka_s[NC * KAP];  // [j][t], theta_j at t = KK
  using SP = SplitPlanes<TW, TH>;
  __shared__ __attribute__((aligned(16))) unsigned u16w[SPLIT ? SP::WORDS : 1];
  __shared__ float wmax[SPLIT ? NT / 64 : 1];


  const int tid = threadIdx.x;
  const Problem pb = a.pb;
  const TileDesc td = a.tiles[blockIdx.x];
  const ImageDesc im = a.images[td.image];
  const int H = im.H, W = im.W, bc = pb.bc, model = pb.model;
  const float lam1 = im.lam1, lam2 = im.lam2;
  const bool logm = model != IDIV;
  const int x0 = td.x0, y0 = td.y0;

  // taps of the next chunk, fetched one chunk ahead (chunk 0: before stage 1) so that their HBM latency
  // is hidden behind the work in between
  constexpr bool PREFETCH = true;
  constexpr int KF_PT = (KF_N + NT - 1) / NT, KA_PT = (NC * KAP + NT - 1) / NT;
  float kfr[KF_PT], kar[KA_PT];
  auto fetch_taps = [&](int cn) {
#pragma unroll
    for (int q = 0; q < KF_PT; ++q) {
      const int t = tid + q * NT;
      if constexpr (SPLIT)
        kfr[q] = t < KF_N ? __uint_as_float(a.kf16[(size_t)(cn / NC) * F16_OPS + t]) : 0.0f;
      else
        kfr[q] = t < KF_N ? a.kf[(size_t)cn * KK + t] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < KA_PT; ++q) {
      const int t = tid + q * NT, j = t / KAP, tt = t - j * KAP;
      kar[q] = t < NC * KAP && tt < KK ? a.ka[(size_t)(cn + j) * KK + tt]
                                       : (t < NC * KAP && tt == KK ? a.theta[cn + j] : 0.0f);
    }
  };
  if constexpr (PREFETCH) fetch_taps(0);

  // split engine: live / own bits of this lane's forward passes, the same in every chunk
  unsigned pmask = 0u;
  bool have_pmask = false;
  const float* xc;
  const float* xp = nullptr;
  const float* gc = nullptr;
  float* xo = nullptr;
  float* go;
  float alpha = 0.0f;
  if (a.mode == MODE_TRIAL) {
    const DevState* st = a.st + td.image;
    __shared__ DevState s_dec;
    if (a.decide_prev) {
      // the decision on the previous trial of this image: every workgroup of the image reduces the same
      // partials in the same fixed order and so takes the same decision (no inter-workgroup sync).  The
      // state is fetched together with the partials.
      // the reduction is image_totals, the one of decide_kernel: the same totals, hence the same decision
      if (tid == 0) s_dec = *st;
      double tot[5];
      image_totals(a.part_in, im.tile0, im.ntiles, red, tot);
      // the other waves form their pass masks while thread 0 decides
      if constexpr (SPLIT) {
        pmask = patch_masks<TW, TH, NT / 64>(tid >> 6, tid & 15, y0, x0, H, W, bc == PERIODIC);
        have_pmask = true;
      }
      if (tid == 0) {
        const bool writer = (int)blockIdx.x == im.tile0;
        if (s_dec.pending && !s_dec.done) {
#pragma unroll
          for (int k = 0; k < PART_COLS; ++k) s_dec.sums[k] = k < 5 ? tot[k] : 0.0;
          decide_step(s_dec, tot, pb, writer ? a.stats + (size_t)td.image * a.stats_rows * STAT_COLS : nullptr);
        }
        s_dec.pending = s_dec.done ? 0 : 1;   // this launch runs the next trial unless the image is done
        if (writer) a.st_out[td.image] = s_dec;
      }
      __syncthreads();
      st = &s_dec;
    }
    if (st->done) return;
    alpha = (float)st->alpha;
    xc = pick3(st->icur, a.xr0, a.xr1, a.xr2) + im.off;
    xp = pick3(st->iprev, a.xr0, a.xr1, a.xr2) + im.off;
    xo = pick3(st->icand, a.xr0, a.xr1, a.xr2) + im.off;
    gc = pick2(st->gcur, a.gr0, a.gr1) + im.off;
    go = pick2(st->gcand, a.gr0, a.gr1) + im.off;
  } else {
    xc = a.x_in + im.off;
    go = a.g_out + im.off;
  }
  // chunk 0's taps go to LDS now (stage 1 does not read them): their loads, issued at the start, have landed
  // with the prologue's, and a store at the first chunk would also wait for stage 1's global stores.  Chunk 1's
  // taps are fetched next, into the same registers.
  auto stage_taps = [&]() {
#pragma unroll
    for (int q = 0; q < KF_PT; ++q)
      if (tid + q * NT < KF_N) kf_s[tid + q * NT] = kfr[q];
#pragma unroll
    for (int q = 0; q < KA_PT; ++q)
      if (tid + q * NT < NC * KAP) ka_s[tid + q * NT] = kar[q];
  };
  if constexpr (PREFETCH) {
    stage_taps();
    if (NC < pb.nf) fetch_taps(NC);
  }
  const float* __restrict__ f = a.f + im.off;
  const bool fold = UNF != FWD_HALF && bc == SYMMETRIC && (y0 < R || y0 + TH > H - R || x0 < R || x0 + TW > W - R);
  // every R3 position (tile + 3) in the image: z needs no mask, every tile position is an own one
  const bool all_in = y0 >= R && y0 + TH + R <= H && x0 >= R && x0 + TW + R <= W;

  double accF = 0.0, accG = 0.0, accS1 = 0.0, accS2 = 0.0, accM = 0.0;
  float usc = 1.0f;   // split-FP16 engine: the tile's scale 2^E of u


  // ---- stage 1: step + prox on tile + 6 halo -> u6 (ADJ_HALF: u+ = e^{x+} on the tile only, x+
  // as written by FWD_HALF)
  if constexpr (UNF == ADJ_HALF) {
    const float* xs = a.mode == MODE_TRIAL ? xo : xc;
    for (int idx = tid; idx < TH * TW; idx += NT) {
      const int i = idx / TW, jx = idx - i * TW, py = y0 + i, px = x0 + jx;
      if (py < H && px < W) {
        const float xn = xs[(size_t)py * W + px];
        u6[(i + 2 * R) * W6 + jx + 2 * R] = logm ? fast_exp(xn) : xn;
      }
    }
    // the halves after the last strip, which no chunk writes, read by the matrix-core adjoint's last rows
    // (k >= 154) against zero taps: zeros, as in the fused kernel
    if constexpr (ZSPLIT)
      if (tid < 4) reinterpret_cast<unsigned*>(zp)[NC * ZS::FILTER_H / 2 + tid] = 0u;
  } else {
    // the positions of this thread, two at a time: their loads first (invalid positions read pixel 0
    // and are discarded), so that the HBM latency of the block's inputs is paid once per batch
    constexpr int P1 = 2;
    float umx = 0.0f;   // largest |u| of this thread (split-FP16 engine)
#pragma unroll 1
    for (int b0 = tid; b0 < H6 * W6; b0 += P1 * NT) {
    int ps[P1];
    bool pv[P1];
    float fv[P1], xv[P1], xpv[P1], gv[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      const int idx = b0 + k * NT;
      const int r = idx / W6, c = idx - r * W6;
      const int sy = bmap(y0 - 2 * R + r, H, bc), sx = bmap(x0 - 2 * R + c, W, bc);
      pv[k] = idx < H6 * W6 && sy >= 0 && sx >= 0;
      ps[k] = pv[k] ? sy * W + sx : 0;
      fv[k] = f[ps[k]];
      xv[k] = xc[ps[k]];
      if (a.mode == MODE_TRIAL) {
        xpv[k] = xp[ps[k]];
        gv[k] = gc[ps[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) {
      const int idx = b0 + k * NT;
      if (idx >= H6 * W6) break;
      const int r = idx / W6, c = idx - r * W6;
      const int gy = y0 - 2 * R + r, gx = x0 - 2 * R + c;
      float uval = 0.0f;
      if (pv[k]) {
        const bool own = r >= 2 * R && r < 2 * R + TH && c >= 2 * R && c < 2 * R + TW && gy < H && gx < W;
        float xn;
        if (a.mode == MODE_TRIAL) {
          const float xh = xv[k] - alpha * gv[k] + pb.beta * (xv[k] - xpv[k]);
          xn = prox_pixel(xh, fv[k], alpha, model, lam1, lam2, pb.newton_iters, pb.prox_method);
          uval = logm ? fast_exp(xn) : xn;
          if (own) {
            xo[ps[k]] = xn;
            const float d = xn - xv[k], m = xv[k] - xpv[k];
            accS1 += (double)(gv[k] * d);
            accS2 += (double)(d * d);
            accM += (double)(m * m);
            accG += (double)data_term(xn, uval, fv[k], model, lam1, lam2);
          }
        } else {
          xn = xv[k];
          uval = logm ? fast_exp(xn) : xn;
          if (own) accG += (double)data_term(xn, uval, fv[k], model, lam1, lam2);
        }
      }
      u6[idx] = uval;
      if constexpr (SPLIT) {
        umx = fmaxf(umx, fabsf(uval));
        split_store<TW, TH>(u16w, r, c, uval);
      }
    }
    }
    if constexpr (SPLIT) {
      // the planes were written unscaled (E = 0); the zero padding, and this wave's largest |u| for the
      // check after the barrier below
      _Float16* h = reinterpret_cast<_Float16*>(u16w);
      constexpr int COPY_H = 2 * SP::COPY1, ROW_H = 2 * SP::ROW_W;
      constexpr int NP0 = SP::COLS - W6, NPR = 2 * (2 * NP0 + 1), NLAST = 4 * SP::COLS;
      for (int i = tid; i < H6 * NPR + NLAST; i += NT) {
        int cp, row, part, col;
        if (i < H6 * NPR) {
          row = i / NPR;
          int q = i - row * NPR;
          part = q & 1;
          q >>= 1;
          cp = q >= NP0;
          col = cp ? W6 - 1 + (q - NP0) : W6 + q;
        } else {
          int q = i - H6 * NPR;
          cp = q / (2 * SP::COLS);
          q -= cp * 2 * SP::COLS;
          part = q / SP::COLS;
          col = q - part * SP::COLS;
          row = H6;
        }
        h[cp * COPY_H + row * ROW_H + part * SP::COLS + col] = (_Float16)0.0f;
      }
      if constexpr (ZSPLIT)   // the halves after the last strip, read by the last rows' k >= 154 (zero taps)
        if (tid < 4) reinterpret_cast<unsigned*>(zp)[NC * ZS::FILTER_H / 2 + tid] = 0u;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) umx = fmaxf(umx, __shfl_xor(umx, o));
      if ((tid & 63) == 0) wmax[tid >> 6] = umx;
    }
  }

  // ---- fold tiles: clear the fold partials and count the fold items, filter index fastest: blocks of
  // FB positions along each live edge (y edges: the TW columns; x edges: the TH rows), then single
  // positions for the corner rows of the x edges whose target row lies in the tile
  const bool e_ylo = fold && y0 == 0, e_yhi = fold && y0 + TH >= H - (R - 1);
  const bool e_xlo = fold && x0 == 0, e_xhi = fold && x0 + TW >= W - (R - 1);
  const int c_lo = y0 == 0 ? R : 0;                               // low-corner rows i = 0..2
  const int c_h0 = max(0, H - y0 - TH), c_h1 = min(R - 1, H - 1 - y0);  // high-corner rows i
  const int c_hn = e_yhi ? max(0, c_h1 - c_h0 + 1) : 0;
  constexpr int FB = 2;                                 // positions per block item
  static_assert(TW % FB == 0 && TH % FB == 0, "fold blocks tile the edges");
  const int ncr = c_lo + c_hn;                          // corner rows per x edge
  const int f_y1 = e_ylo ? NC * (TW / FB) : 0;          // item starts: y-high blocks, x-low blocks,
  const int f_x0 = f_y1 + (e_yhi ? NC * (TW / FB) : 0); // x-high blocks, x-low corner rows, x-high
  const int f_x1 = f_x0 + (e_xlo ? NC * (TH / FB) : 0); // corner rows; and the item count
  const int f_c0 = f_x1 + (e_xhi ? NC * (TH / FB) : 0);
  const int f_c1 = f_c0 + (e_xlo ? NC * ncr : 0);
  const int n_items = f_c1 + (e_xhi ? NC * ncr : 0);
  if (fold)
    for (int i = tid; i < NSLOT * R * NC; i += NT) fpart[i] = 0.0f;

  // forward positions of this thread (fixed across chunks)
  int fbase[PPT];      // u6 offset of the window's top-left sample, or -1 when the slot is empty
  int zofs[PPT];       // z-plane offset of the position
  bool flive[PPT], fown[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    int idx = tid + k * NT;
    int r = idx / W3, c = idx - r * W3;
    int gy = y0 - R + r, gx = x0 - R + c;
    bool inimg = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
    fbase[k] = idx < PLANE3 ? r * W6 + c : -1;
    zofs[k] = r * ZW + c;
    flive[k] = idx < PLANE3 && (inimg || bc == PERIODIC);
    fown[k] = idx < PLANE3 && inimg && r >= R && r < R + TH && c >= R && c < R + TW;
  }

  // adjoint mapping: group grp takes FPG filters of each chunk; thread owns a BR x BC block
  const int grp = __builtin_amdgcn_readfirstlane(tid / GT);  // wave-uniform (GT % 64 == 0)
  const int lt = tid - grp * GT;
  const int col0 = (lt % (TW / BC)) * BC;
  const int row0 = (lt / (TW / BC)) * BR;
  float acc[BR][BC];
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int j = 0; j < BC; ++j) acc[i][j] = 0.0f;

  __syncthreads();
  if constexpr (SPLIT) {
    if constexpr (UNF != ADJ_HALF) {
      // the tile's scale 2^E: none (E = 0) when the largest |u| lies in [2^-4, 2^14), where the heads stay
      // below 2^14 and the absolute resolution of the split (2^-36) is far below the FP32 rounding of the
      // largest terms; else largest |u| / 2^E in [2^13, 2^14), and the planes are written again
      float m = 0.0f;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) m = fmaxf(m, wmax[w]);
      if (!(m >= 0.0625f && m < 16384.0f)) {
        const int E = min(max(((__float_as_int(m) >> 23) & 0xff) - 127 - 13, -100), 100);
        const float isc = __int_as_float((127 - E) << 23);
        for (int idx = tid; idx < H6 * W6; idx += NT) {
          const int r = idx / W6, c = idx - r * W6;
          split_store<TW, TH>(u16w, r, c, u6[idx] * isc);
        }
        usc = __int_as_float((127 + E) << 23);
        __syncthreads();
      }
    }
  }

  if constexpr (SPLIT)
    if (!have_pmask) pmask = patch_masks<TW, TH, NT / 64>(tid >> 6, tid & 15, y0, x0, H, W, bc == PERIODIC);

  // matrix-core adjoint (ZSPLIT): this wave's filter of each chunk on the NB output blocks of the tile, summed
  // over the chunks in gacc
  constexpr int NBZ = ZSPLIT ? ZS::NB : 1;
  floatx4 gacc[NBZ];
#pragma unroll
  for (int q = 0; q < NBZ; ++q) gacc[q] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index (uniform)
  const int ln = tid & 15, lkb = (tid >> 4) & 3;            // lane (n, kb) of the 16 x 16 x 32 operands

  const int nf = pb.nf;
  for (int c0 = 0; c0 < nf; c0 += NC) {
    const int ncur = min(NC, nf - c0);
    if constexpr (PREFETCH) {
      if (c0 > 0) {   // chunk 0 was staged before stage 1
        stage_taps();
        if (c0 + NC < nf) fetch_taps(c0 + NC);
      }
    } else {
      for (int t = tid; t < KK * NC; t += NT) kf_s[t] = a.kf[(size_t)c0 * KK + t];
      for (int t = tid; t < NC * KAP; t += NT) {
        const int j = t / KAP, tt = t - j * KAP;
        ka_s[t] = tt < KK ? a.ka[(size_t)(c0 + j) * KK + tt] : (tt == KK ? a.theta[c0 + j] : 0.0f);
      }
    }
    __syncthreads();
    if constexpr (UNF == ADJ_HALF) {
      // ---- z of this chunk from HBM on the tile + 3 halo (zero off the image, wrapped when periodic);
      // the positions of this thread are the ones of the VALU forward (fbase / zofs / flive)
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (fbase[k] < 0) continue;
        const int idx = tid + k * NT, r = idx / W3, c = idx - r * W3;
        int gy = y0 - R + r, gx = x0 - R + c;
        gy = gy < 0 ? gy + H : (gy >= H ? gy - H : gy);
        gx = gx < 0 ? gx + W : (gx >= W ? gx - W : gx);
        const float* src = a.zbuf + (size_t)c0 * a.zstride + im.off + (size_t)gy * W + gx;
        float zv[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) zv[j] = flive[k] && j < ncur ? src[(size_t)j * a.zstride] : 0.0f;
        if constexpr (ZSPLIT) {
          // the strips of the fused BF16 kernel (the same rounding of the same FP32 z, so both paths give the
          // same bits): strip 0 for the columns < 22, strip 1 for the columns >= 16
          __bf16* zh = reinterpret_cast<__bf16*>(zp) + r * ZS::W + c;
#pragma unroll
          for (int j = 0; j < NC; ++j) {
            const __bf16 hv = (__bf16)zv[j];
            if (c < ZS::W) zh[j * ZS::FILTER_H] = hv;
            if (c >= 16) zh[j * ZS::FILTER_H + ZS::STRIP_H - 16] = hv;
          }
        } else {
#pragma unroll
          for (int j = 0; j < NC; ++j) zp[j * PLANE + zofs[k]] = zv[j];
        }
      }
    } else if constexpr (FWD == FWD_MFMA_F32 || SPLIT) {
      // ---- stage 2 (matrix cores): per group of 16 consecutive R3 positions,
      // Y^T[16 filters x 16 positions] = Kflip^T[16 x taps] . X[taps x 16 positions].  FP32 engine:
      // twelve v_mfma_f32_16x16x4f32 over taps 0..47 and the last tap (48) on the VALU; lane (m = lane % 16,
      // k = lane / 16) holds the A value Kflip[filter m][tap 4s + k] and the B value u6 at tap 4s + k of
      // position m.  Split-FP16 engine: the operands of ForwardOps<FWD_MFMA_F16X>, staged per lane in
      // kf_s.  Either way the result lands as y for position m, filters 4k .. 4k + 3.
      const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lm = lane & 15, lk = lane >> 4;
      ForwardOps<FWD> ops;
      if constexpr (FWD == FWD_MFMA_F32) {
        constexpr int NS4 = KK / 4;                  // 12 MFMA steps of 4 taps; KK = 4 NS4 + 1
#pragma unroll
        for (int s = 0; s < NS4; ++s) {
          const int t = 4 * s + lk;
          ops.a[s] = kf_s[t * NC + lm];
          // taps 4s + k and 4(s + 7) + k are 28 = 4 KS apart: 4 rows of u6 in every lane, so that the
          // loads of steps s and s + 7 share an address register (the difference is an immediate)
          ops.toff[s] = s < KS ? (t / KS) * W6 + (t % KS) : ops.toff[s - KS] + 4 * W6;
        }
        ops.klast = *reinterpret_cast<const float4*>(kf_s + (KK - 1) * NC + 4 * lk);  // tap 48, filters 4k..
      } else {
        const u32x4* src = reinterpret_cast<const u32x4*>(kf_s) + lane * 4;   // [step][head, tail]
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          ops.hi[s] = __builtin_bit_cast(half8, src[2 * s]);
          ops.lo[s] = __builtin_bit_cast(half8, src[2 * s + 1]);
        }
        ops.sc = usc;
        ops.sclo = usc * (1.0f / 4096.0f);
      }
      float thl[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) thl[j] = ka_s[(4 * lk + j) * KAP + KK] * 0.6931471805599453f;   // theta ln 2
      // one position group per pass: with four waves per SIMD the other waves' chains fill the
      // matrix pipe while this one waits for its predecessor
      float* zb = UNF == FWD_HALF ? a.zbuf + (size_t)c0 * a.zstride + im.off : nullptr;
      float ef;
      if (SPLIT && usc == 1.0f)
        ef = all_in ? mfma_forward_chunk<TW, TH, NC, NT / 64, UNF, true, FWD, true>(
                          u6, u16w, zp, ops, thl, wave, lm, lk, y0, x0, H, W, bc == PERIODIC, zb, a.zstride, ncur, pmask)
                    : mfma_forward_chunk<TW, TH, NC, NT / 64, UNF, false, FWD, true>(
                          u6, u16w, zp, ops, thl, wave, lm, lk, y0, x0, H, W, bc == PERIODIC, zb, a.zstride, ncur, pmask);
      else
        ef = all_in ? mfma_forward_chunk<TW, TH, NC, NT / 64, UNF, true, FWD>(
                          u6, u16w, zp, ops, thl, wave, lm, lk, y0, x0, H, W, bc == PERIODIC, zb, a.zstride, ncur, pmask)
                    : mfma_forward_chunk<TW, TH, NC, NT / 64, UNF, false, FWD>(
                          u6, u16w, zp, ops, thl, wave, lm, lk, y0, x0, H, W, bc == PERIODIC, zb, a.zstride, ncur, pmask);
      accF += (double)ef;
    } else {
      // ---- stage 2: forward bank on tile + 3 halo; one row of taps of 8 filters (in SGPRs) per pass
      float y[PPT][NC];
  #pragma unroll
      for (int k = 0; k < PPT; ++k)
  #pragma unroll
        for (int j = 0; j < NC; ++j) y[k][j] = 0.0f;
      constexpr int NH = NC / 8;
  #pragma unroll 1
      for (int ta = 0; ta < KS; ++ta) {
  #pragma unroll
        for (int h = 0; h < NH; ++h) {
          float kr[KS * 8];
  #pragma unroll
          for (int tb = 0; tb < KS; ++tb) {
            const float4* src = reinterpret_cast<const float4*>(kf_s + (ta * KS + tb) * NC + h * 8);
            float4 p0 = src[0], p1 = src[1];
            kr[tb * 8 + 0] = p0.x; kr[tb * 8 + 1] = p0.y; kr[tb * 8 + 2] = p0.z; kr[tb * 8 + 3] = p0.w;
            kr[tb * 8 + 4] = p1.x; kr[tb * 8 + 5] = p1.y; kr[tb * 8 + 6] = p1.z; kr[tb * 8 + 7] = p1.w;
          }
  #pragma unroll
          for (int k = 0; k < PPT; ++k) {
            if (fbase[k] < 0) continue;
            float wrow[KS];
  #pragma unroll
            for (int tb = 0; tb < KS; ++tb) wrow[tb] = u6[fbase[k] + ta * W6 + tb];
  #pragma unroll
            for (int tb = 0; tb < KS; ++tb)
  #pragma unroll
              for (int j = 0; j < 8; ++j) y[k][h * 8 + j] = fmaf(kr[tb * 8 + j], wrow[tb], y[k][h * 8 + j]);
          }
        }
      }
      // rho' into the z planes (zero off the image unless periodic), theta * rho summed over the tile
  #pragma unroll
      for (int k = 0; k < PPT; ++k) {
        if (fbase[k] < 0) continue;
        float e = 0.0f;
  #pragma unroll
        for (int j = 0; j < NC; ++j) {
          const float th = ka_s[j * KAP + KK];   // theta_j (zero past the bank)
          float den = fmaf(y[k][j], y[k][j], 1.0f);
          float z = y[k][j] * fast_rcp(den);
          zp[j * PLANE + zofs[k]] = flive[k] ? z : 0.0f;
          if (UNF == FWD_HALF && fown[k] && j < ncur) {
            const int idx = tid + k * NT, r = idx / W3, c = idx - r * W3;
            a.zbuf[(size_t)(c0 + j) * a.zstride + im.off + (size_t)(y0 - R + r) * W + (x0 - R + c)] = z;
          }
          e = fmaf(th, fast_log(den), e);
        }
        if (fown[k]) accF += (double)e;
      }
    }
    // matrix-core adjoint: the B operands (Toeplitz tap rows) of this wave's filter for every K step, fetched
    // before the barrier so that their latency overlaps the wait; lane (n, kb) of step s takes
    // T[32 s + 8 kb - n .. + 7] from copy n & 1
    constexpr int KST = ZSPLIT ? ZS::KSTEPS : 1;
    u32x4 bw[KST];
    if constexpr (ZSPLIT) {
      if (wv < ncur) {
        const unsigned* tb = a.kb16 + (size_t)(c0 + wv) * KB16_W + (ln & 1) * KB16_COPY + ((16 - ln - (ln & 1)) >> 1) +
                             4 * lkb;
#pragma unroll
        for (int st = 0; st < KST; ++st) {
          const unsigned* th = tb + 16 * st;
          bw[st] = u32x4{th[0], th[1], th[2], th[3]};
        }
      }
    }
    __syncthreads();

    // ---- stage 3: adjoint bank.
    // ZSPLIT: wave wv takes filter wv of the chunk on every 16 x 16 output block (ZStrips): per K step one
    // v_mfma_f32_16x16x32_bf16, A = the block's z strip rows, B = the Toeplitz taps; FP32 sums in gacc.
    if constexpr (ZSPLIT) {
      if (wv < ncur) {
        const __bf16* zw = reinterpret_cast<const __bf16*>(zp) + wv * ZS::FILTER_H + ln * ZS::W + 8 * lkb;
#pragma unroll
        for (int st = 0; st < KST; ++st) {
          const bf16x8 bb = __builtin_bit_cast(bf16x8, bw[st]);
#pragma unroll
          for (int q = 0; q < NBZ; ++q) {
            const int rb = q / ZS::NS, sb = q - rb * ZS::NS;
            const unsigned* pa = reinterpret_cast<const unsigned*>(zw + sb * ZS::STRIP_H + 16 * rb * ZS::W + 32 * st);
            const bf16x8 ab = __builtin_bit_cast(bf16x8, u32x4{pa[0], pa[1], pa[2], pa[3]});
            gacc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, gacc[q], 0, 0, 0);
          }
        }
      }
    }
    // VALU: per filter of the group the BR x BC block of this thread from a (BR+6) x (BC+6) window in
    // registers.  Then, on fold tiles, the fold items of the chunk.
#pragma unroll 1
    for (int jj = 0; jj < (UNF == FWD_HALF || ZSPLIT ? 0 : FPG); ++jj) {
      const int j = grp * FPG + jj;
      if (j >= ncur) break;
      float kt[KAP];
#pragma unroll
      for (int t = 0; t < KAP; t += 4) {
        float4 q4 = *reinterpret_cast<const float4*>(ka_s + j * KAP + t);
        kt[t] = q4.x; kt[t + 1] = q4.y; kt[t + 2] = q4.z; kt[t + 3] = q4.w;
      }
      const float* zplane = zp + j * PLANE;
      const float* zb = zplane + row0 * ZW + col0;
      // stream the (BR+6) x (BC+6) window one row at a time; row q feeds output rows q - ta
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        float wrow[WC];
        if constexpr (WIN4) {
#pragma unroll
          for (int s = 0; s + 4 <= WC; s += 4) {
            const float4 v4 = *reinterpret_cast<const float4*>(zb + q * ZW + s);
            wrow[s] = v4.x;
            wrow[s + 1] = v4.y;
            wrow[s + 2] = v4.z;
            wrow[s + 3] = v4.w;
          }
#pragma unroll
          for (int s = WC / 4 * 4; s < WC; s += 2) {
            const float2 v2 = *reinterpret_cast<const float2*>(zb + q * ZW + s);
            wrow[s] = v2.x;
            wrow[s + 1] = v2.y;
          }
        } else {
#pragma unroll
          for (int s = 0; s < WC; s += 2) {
            const float2 v2 = *reinterpret_cast<const float2*>(zb + q * ZW + s);
            wrow[s] = v2.x;
            wrow[s + 1] = v2.y;
          }
        }
#pragma unroll
        for (int ta = 0; ta < KS; ++ta) {
          const int i = q - ta;
          if (i < 0 || i >= BR) continue;
#pragma unroll
          for (int tb = 0; tb < KS; ++tb)
#pragma unroll
            for (int jx = 0; jx < BC; ++jx) acc[i][jx] = fmaf(kt[ta * KS + tb], wrow[jx + tb], acc[i][jx]);
        }
      }
    }
    // the fold items of this thread (all threads take part; a pass of its own after the regular
    // blocks, whose window registers are dead by then).  Each item owns its partials.
    if (fold) {
#pragma unroll 1
      for (int it = tid; it < n_items; it += NT) {
        if (it < f_x0) {
          // y edge block, tile columns p0 .. p0 + FB - 1: z lines are plane rows, taps run along tap rows
          const bool lo = it < f_y1;
          const int loc = it - (lo ? 0 : f_y1), j = loc & (NC - 1), p0 = (loc / NC) * FB;
          if (j >= ncur) continue;
          float* out = fpart + ((lo ? 0 : TW) + p0) * R * NC + j;
          const int zrow = lo ? R : H - 1 - y0 + R;   // plane row of the edge line
          if constexpr (ZSPLIT) {
            // the FB + 6 columns p0 .. p0 + FB + 5 lie in strip 0 when p0 < 16, else in strip 1
            const int sb = p0 >= 16;
            const __bf16* zl = reinterpret_cast<const __bf16*>(zp) + j * ZS::FILTER_H + sb * ZS::STRIP_H +
                               zrow * ZS::W + p0 - 16 * sb;
            if (lo)
              fold_block<FB, NC, 1, KS>(ZLines<1, ZS::W, true>{zl}, ka_s + j * KAP + (R + 1) * KS, out);
            else
              fold_block<FB, NC, 1, -KS>(ZLines<1, -ZS::W, true>{zl}, ka_s + j * KAP + (R - 1) * KS, out);
          } else {
            if (lo)
              fold_block_y<FB, NC, true>(zp + j * PLANE + zrow * ZW + p0, ZW, ka_s + j * KAP, out);
            else
              fold_block_y<FB, NC, false>(zp + j * PLANE + zrow * ZW + p0, -ZW, ka_s + j * KAP, out);
          }
        } else if (it < f_c0) {
          // x edge block, tile rows p0 .. p0 + FB - 1: z lines are plane columns, taps run down tap columns
          const bool lo = it < f_x1;
          const int loc = it - (lo ? f_x0 : f_x1), j = loc & (NC - 1), p0 = (loc / NC) * FB;
          if (j >= ncur) continue;
          float* out = fpart + (2 * TW + (lo ? 0 : NPX) + p0) * R * NC + j;
          const int zcol = lo ? R : W - 1 - x0 + R;   // plane column of the edge line
          if constexpr (ZSPLIT) {
            // the three lines zcol, zcol -+ 1, zcol -+ 2 lie in strip 0 when zcol <= 21, else in strip 1
            const int sb = zcol > 21;
            const __bf16* zl = reinterpret_cast<const __bf16*>(zp) + j * ZS::FILTER_H + sb * ZS::STRIP_H +
                               p0 * ZS::W + zcol - 16 * sb;
            if (lo)
              fold_block<FB, NC, KS, 1>(ZLines<ZS::W, 1, true>{zl}, ka_s + j * KAP + R + 1, out);
            else
              fold_block<FB, NC, KS, -1>(ZLines<ZS::W, -1, true>{zl}, ka_s + j * KAP + R - 1, out);
          } else {
            if (lo)
              fold_block_x<FB, NC, true>(zp + j * PLANE + p0 * ZW, ZW, zcol, ka_s + j * KAP, out);
            else
              fold_block_x<FB, NC, false>(zp + j * PLANE + p0 * ZW, ZW, zcol, ka_s + j * KAP, out);
          }
        } else {
          // a corner row (-1 - i or H + i) of an x edge: window rows outside the plane are off the image
          // (rows < 0 for the low corners, >= H for the high ones); they read the plane's first / last
          // row, which is off the image too
          const int e = it < f_c1 ? 2 : 3;
          const int loc = it - (e == 2 ? f_c0 : f_c1), j = loc & (NC - 1), q = loc / NC;
          if (j >= ncur) continue;
          const int zc0 = e == 2 ? R : W - 1 - x0 + R;            // plane column of the edge line
          const int zls = e == 2 ? 1 : -1;
          const float* kb = ka_s + j * KAP + (e == 2 ? R + 1 : R - 1);
          const int kls = e == 2 ? 1 : -1;
          const int gy = q < c_lo ? -1 - q : H + c_h0 + q - c_lo;
          const int slot = 2 * TW + (e - 2) * NPX + (q < c_lo ? TH + q : TH + R + c_h0 + q - c_lo);
          const int prow = gy - y0;                              // plane row of window row 0
          float Z[R][KS], K[R][KS];
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            const int pr = min(max(prow + t, 0), H3 - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if constexpr (ZSPLIT) {
                const int sb = zc0 > 21;   // the three lines share a strip (as for the x-edge blocks)
                Z[r][t] = (float)reinterpret_cast<const __bf16*>(zp)[j * ZS::FILTER_H + sb * ZS::STRIP_H + pr * ZS::W +
                                                                      zc0 - 16 * sb + r * zls];
              } else {
                Z[r][t] = zp[j * PLANE + zc0 + pr * ZW + r * zls];
              }
              K[r][t] = kb[r * kls + t * KS];
            }
          }
          float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
#pragma unroll
          for (int t = 0; t < KS; ++t) {
            v0 = fmaf(K[0][t], Z[0][t], v0);
            v0 = fmaf(K[1][t], Z[1][t], v0);
            v0 = fmaf(K[2][t], Z[2][t], v0);
            v1 = fmaf(K[1][t], Z[0][t], v1);
            v1 = fmaf(K[2][t], Z[1][t], v1);
            v2 = fmaf(K[2][t], Z[0][t], v2);
          }
          float* fo = fpart + slot * R * NC + j;
          fo[0] += v0;
          fo[NC] += v1;
          fo[2 * NC] += v2;
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: combine groups and mirror terms in a fixed order, chain rule, store
  if constexpr (UNF == FWD_HALF) {
    double v[5] = {accF, accG, accS1, accS2, accM};
    block_partials<NT, 5>(v, red, a.partials);
    return;
  }
  float* gsum = zp;                       // [NG][TH][TW]
  if constexpr (ZSPLIT) {
    // lane (n, kb) of block (rb, sb) holds rows 16 rb + 4 kb + i, column 16 sb + n
#pragma unroll
    for (int q = 0; q < NBZ; ++q) {
      const int rb = q / ZS::NS, sb = q - rb * ZS::NS;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        gsum[wv * TH * TW + (16 * rb + 4 * lkb + i) * TW + 16 * sb + ln] = gacc[q][i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < BR; ++i)
#pragma unroll
      for (int jx = 0; jx < BC; ++jx) gsum[grp * TH * TW + (row0 + i) * TW + col0 + jx] = acc[i][jx];
  }
  __syncthreads();
  for (int idx = tid; idx < TH * TW; idx += NT) {
    int i = idx / TW, jx = idx - i * TW;
    int py = y0 + i, px = x0 + jx;
    if (py >= H || px >= W) continue;
    float g = 0.0f;
#pragma unroll
    for (int q = 0; q < NG; ++q) g += gsum[q * TH * TW + idx];
    if (fold) {
      // mirror terms of this pixel (edges, then corners), each summed over the NC filter partials
      // in filter order; a pixel of an image 4 or 5 wide lies within 3 of both opposite edges
      const int dyl = py, dyh = H - 1 - py, dxl = px, dxh = W - 1 - px;
      const int xl = 2 * TW, xh = 2 * TW + NPX;
      auto add = [&](int slot, int d) {
        const float* fp = fpart + (slot * R + d) * NC;
#pragma unroll
        for (int jj = 0; jj < NC; ++jj) g += fp[jj];
      };
      if (dyl < R) add(jx, dyl);
      if (dyh < R) add(TW + jx, dyh);
      if (dxl < R) add(xl + i, dxl);
      if (dxh < R) add(xh + i, dxh);
      if (dxl < R && dyl < R) add(xl + TH + dyl, dxl);
      if (dxl < R && dyh < R) add(xl + TH + R + dyh, dxl);
      if (dxh < R && dyl < R) add(xh + TH + dyl, dxh);
      if (dxh < R && dyh < R) add(xh + TH + R + dyh, dxh);
    }
    if (logm) g *= u6[(i + 2 * R) * W6 + jx + 2 * R];
    go[(size_t)py * W + px] = g;
  }

  if constexpr (UNF == FUSED) {
    double v[5] = {accF, accG, accS1, accS2, accM};
    block_partials<NT, 5>(v, red, a.partials);
  }
}

}  // namespace foe
