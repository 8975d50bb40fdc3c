// Fused FoE trial kernel, VALU direct-convolution engine.
//
// One workgroup owns one TH x TW output tile and runs, entirely on chip:
//   1. the inertial step and the pointwise prox on the tile + 6-pixel halo
//      (x+ = prox_{aG}(x - a grad F(x) + b (x - x_prev)), Sec. II-C, eq. (fplusg)),
//      then u+ = e^{x+} (log models) into LDS;
//   2. per chunk of NC filters: the forward bank y_i = K_i u+ on the tile + 3 halo,
//      z_i = theta_i rho'(y_i) into LDS, and theta_i rho(y_i) summed over the tile
//      (F(x+), Sec. II-A, eq. (FOEmodel));
//   3. per chunk: the adjoint bank sum_i K_i^T z_i on the tile (correlation with k_i,
//      Sec. II-C), plus the mirror terms of the SYMMETRIC boundary map;
//   4. the chain rule grad_w F = u .* sum_i K_i^T z_i, written as the gradient at x+
//      for the next iteration (speculative: used only if the trial is accepted),
//      and per-block partial sums {F(x+), G(x+), <grad F(x), d>, |d|^2, |x - x_prev|^2}.
// In EVAL mode stage 1 is the identity (x+ = x_in): F, G and grad F at x_in.
#pragma once
#include "device_math.hpp"

namespace foe {

enum FusedMode { MODE_TRIAL = 0, MODE_EVAL = 1 };
enum ForwardEngine { FWD_VALU = 0, FWD_MFMA_F32 = 1, FWD_MFMA_BF16 = 2 };
// Fusion of the gradient: the whole trial in one kernel (FUSED), or split in two launches that
// exchange the 48 z planes through HBM: FWD_HALF runs stages 1-2 (step, prox, forward bank,
// energies) and stores z_i on the tile, ADJ_HALF loads z_i on the tile + 3 halo and runs stage 3
// and the chain rule.
enum Fusion { FUSED = 0, FWD_HALF = 1, ADJ_HALF = 2 };
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct FusedArgs {
  Problem pb;
  const TileDesc* tiles;                // [gridDim.x]
  const ImageDesc* images;
  const float* f;                       // packed planes of all images
  float* xr0; float* xr1; float* xr2;   // x ring (TRIAL), packed
  float* gr0; float* gr1;               // gradient ring (TRIAL), packed
  const float* x_in;                    // EVAL input, packed
  float* g_out;                         // EVAL output, packed
  DevState* st;                         // per-image states
  double* partials;                     // [gridDim.x][PART_COLS]
  const float* kf;                      // forward taps, flipped and chunk-transposed:
                                        //   kf[(c * KK + a * 7 + b) * NC + j] = k_{c*NC+j}[6-a][6-b]
  const float* ka;                      // adjoint taps: ka[i][a][b] = k_i[a][b]
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
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) red[wave * NV + k] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w * NV + threadIdx.x];
    out[(size_t)blockIdx.x * PART_COLS + threadIdx.x] = s;
  }
}

// Fold slots of the SYMMETRIC boundary map: the extended samples q != p with source p, for
// pixels p within 3 of the image border.  Slot layout (TW/TH = tile width/height):
//   [0, 3TW)            y-low   q = (-1-py, px),        py in [0,2]
//   [3TW, 6TW)          y-high  q = (2H-1-py, px),      py in [H-3, H-1]
//   [6TW, 6TW+3TH)      x-low   q = (py, -1-px),        px in [0,2]
//   [6TW+3TH, 6TW+6TH)  x-high  q = (py, 2W-1-px),      px in [W-3, W-1]
//   [6TW+6TH, +36)      corners (y-low|y-high) x (x-low|x-high), 3x3 each
// slot_target() returns the owning pixel p (tile-local) and the extended sample q, or false
// when the slot is empty for this tile.
template <int TW, int TH>
__device__ __forceinline__ bool slot_target(int s, int x0, int y0, int H, int W, int& ply, int& plx, int& qy,
                                            int& qx) {
  int py, px;
  if (s < 6 * TW) {
    int hiy = s >= 3 * TW;
    int ss = hiy ? s - 3 * TW : s;
    int d = ss / TW;
    px = x0 + (ss - d * TW);
    py = hiy ? H - 1 - d : d;
    qy = hiy ? 2 * H - 1 - py : -1 - py;
    qx = px;
  } else if (s < 6 * TW + 6 * TH) {
    int s2 = s - 6 * TW;
    int hix = s2 >= 3 * TH;
    int ss = hix ? s2 - 3 * TH : s2;
    int d = ss / TH;
    py = y0 + (ss - d * TH);
    px = hix ? W - 1 - d : d;
    qx = hix ? 2 * W - 1 - px : -1 - px;
    qy = py;
  } else {
    int s3 = s - 6 * TW - 6 * TH;
    int corner = s3 / 9, rem = s3 - corner * 9;
    int dy = rem / 3, dx = rem - dy * 3;
    int hiy = corner >> 1, hix = corner & 1;
    py = hiy ? H - 1 - dy : dy;
    px = hix ? W - 1 - dx : dx;
    qy = hiy ? 2 * H - 1 - py : -1 - py;
    qx = hix ? 2 * W - 1 - px : -1 - px;
  }
  ply = py - y0;
  plx = px - x0;
  return ply >= 0 && ply < TH && plx >= 0 && plx < TW && py >= 0 && py < H && px >= 0 && px < W;
}

// Tile configuration: TW x TH output tile, NC filters per LDS chunk, NT threads, adjoint
// register blocks of BR x BC outputs per thread (NT / ((TH/BR) (TW/BC)) filter groups).
//
// LDS layout: u6 holds u+ on the tile + 6 halo.  Each z plane holds z_j = theta_j rho'(y_j) on
// the tile + 3 halo (R3), surrounded by a zero frame (3 rows above/below, 4 columns left and
// 4 right), so that the 7x7 windows around the extended samples of the SYMMETRIC fold can be read
// without bounds checks; samples off the image are zero.  The rows 0..4 and columns 0..5 of every
// window lie inside the plane.  Only when the next tile holds 1 or 2 rows (columns) does the window
// of a sample mirrored from the far image edge reach up to 2 rows (1 column) past the plane; those
// samples are off the image, so the fold gives them zero weight and reads an in-plane address.
template <int TW, int TH, int NC, int NT, int BR, int BC, int FWD, int UNF = FUSED>
__global__ __launch_bounds__(NT) void foe_trial_kernel(FusedArgs a) {
  constexpr int W6 = TW + 4 * R, H6 = TH + 4 * R;
  constexpr int W3 = TW + 2 * R, H3 = TH + 2 * R;
  constexpr int PLANE3 = H3 * W3;
  constexpr int ZR = R, ZC = R + 1;               // zero frame: rows above, columns left
  constexpr int W3P = W3 + ZC + R + 1, H3P = H3 + 2 * ZR;  // W3P even for float2 reads
  constexpr int PLANEP = H3P * W3P;
  constexpr int PPT = (PLANE3 + NT - 1) / NT;     // forward positions per thread
  constexpr int GT = (TH / BR) * (TW / BC);       // threads per adjoint group
  constexpr int NG = NT / GT;                     // filter groups
  constexpr int FPG = NC / NG;                    // filters per group per chunk
  constexpr int WR = BR + KS - 1, WC = BC + KS - 1;
  constexpr int NS = 6 * TW + 6 * TH + 36;        // fold slots
  constexpr int SLOTS_PT = (NS + GT - 1) / GT;    // compacted fold slots per thread (per group)
  static_assert(NT % GT == 0 && NC % NG == 0 && GT % 64 == 0 && TH % BR == 0 && TW % BC == 0, "bad tiling");
  static_assert(BC % 2 == 0 && W3P % 2 == 0 && PLANEP % 2 == 0 && ZC % 2 == 0, "adjoint reads float2 pairs");
  static_assert(NC % 8 == 0, "forward passes take 8 filters");
  static_assert(NG * (TH * TW + NS) <= NC * PLANEP, "epilogue does not fit in the z buffer");
  static_assert(NS <= 2 * NT, "fold slot scan covers at most two slots per thread");
  static_assert(FWD == FWD_VALU || NC == 16, "the MFMA forwards take one 16-filter block per chunk");
  constexpr int NGROUP = (PLANE3 + 15) / 16;      // MFMA forward: groups of 16 consecutive positions

  __shared__ float u6[H6 * W6];
  __shared__ __attribute__((aligned(16))) float zp[NC * PLANEP];
  __shared__ double red[(NT / 64) * 5];
  __shared__ int act_off[NS];    // compacted fold slots: z-plane offset of the 7x7 window,
  __shared__ short act_slot[NS]; //                       the slot id
  __shared__ char act_rows[NS];  //                       and the window rows / columns that lie
  __shared__ char act_cols[NS];  //                       inside the z plane (at least 5 / 6)
  __shared__ int wave_cnt[NT / 64];
  // taps of the current chunk, read by broadcast LDS loads so that the FMAs take them from VGPRs
  // (a VALU FMA with an SGPR operand issues at half rate on gfx950)
  constexpr int KAP = 52;                                   // padded adjoint tap stride (16 B rows)
  __shared__ __attribute__((aligned(16))) float kf_s[KK * NC];   // [t][j]
  __shared__ __attribute__((aligned(16))) float ka_s[NC * KAP];  // [j][t]

  const int tid = threadIdx.x;
  const Problem pb = a.pb;
  const TileDesc td = a.tiles[blockIdx.x];
  const ImageDesc im = a.images[td.image];
  const int H = im.H, W = im.W, bc = pb.bc, model = pb.model;
  const float lam1 = im.lam1, lam2 = im.lam2;
  const bool logm = model != IDIV;
  const int x0 = td.x0, y0 = td.y0;

  const float* xc;
  const float* xp = nullptr;
  const float* gc = nullptr;
  float* xo = nullptr;
  float* go;
  float alpha = 0.0f;
  if (a.mode == MODE_TRIAL) {
    const DevState* st = a.st + td.image;
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
  const float* __restrict__ f = a.f + im.off;
  const bool fold = UNF != FWD_HALF && bc == SYMMETRIC && (y0 < R || y0 + TH > H - R || x0 < R || x0 + TW > W - R);

  double accF = 0.0, accG = 0.0, accS1 = 0.0, accS2 = 0.0, accM = 0.0;

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
  } else
  for (int idx = tid; idx < H6 * W6; idx += NT) {
    int r = idx / W6, c = idx - r * W6;
    int gy = y0 - 2 * R + r, gx = x0 - 2 * R + c;
    int sy = bmap(gy, H, bc), sx = bmap(gx, W, bc);
    float uval = 0.0f;
    if (sy >= 0 && sx >= 0) {
      size_t p = (size_t)sy * W + sx;
      bool own = r >= 2 * R && r < 2 * R + TH && c >= 2 * R && c < 2 * R + TW && gy < H && gx < W;
      float fv = f[p];
      float xn;
      if (a.mode == MODE_TRIAL) {
        float xv = xc[p], xpv = xp[p], gv = gc[p];
        float xh = xv - alpha * gv + pb.beta * (xv - xpv);
        xn = prox_pixel(xh, fv, alpha, model, lam1, lam2, pb.newton_iters, pb.prox_method);
        uval = logm ? fast_exp(xn) : xn;
        if (own) {
          xo[p] = xn;
          float d = xn - xv, m = xv - xpv;
          accS1 += (double)(gv * d);
          accS2 += (double)(d * d);
          accM += (double)(m * m);
          accG += (double)data_term(xn, uval, fv, model, lam1, lam2);
        }
      } else {
        xn = xc[p];
        uval = logm ? fast_exp(xn) : xn;
        if (own) accG += (double)data_term(xn, uval, fv, model, lam1, lam2);
      }
    }
    u6[idx] = uval;
  }

  // ---- fold tiles: zero the z planes (frame stays zero) and compact the non-empty fold slots
  int n_act = 0;
  if (fold) {
    float4* z4 = reinterpret_cast<float4*>(zp);
    for (int i = tid; i < NC * PLANEP / 4; i += NT) z4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    bool act[2];
    int off[2], nrow[2], ncol[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int s = tid + h * NT, ply, plx, qy, qx;
      act[h] = s < NS && slot_target<TW, TH>(s, x0, y0, H, W, ply, plx, qy, qx);
      const int wr = qy - y0 + ZR, wc = qx - x0 + ZC;
      off[h] = act[h] ? wr * W3P + wc : 0;
      nrow[h] = min(KS, H3P - wr);
      ncol[h] = min(KS, W3P - wc);
    }
    const int lane = tid & 63, wave = tid >> 6;
    int base = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      unsigned long long m = __ballot(act[h]);
      if (lane == 0) wave_cnt[wave] = __popcll(m);
      __syncthreads();
      int before = 0, total = 0;
      for (int w = 0; w < NT / 64; ++w) {
        int cw = wave_cnt[w];
        before += w < wave ? cw : 0;
        total += cw;
      }
      int pos = base + before + __popcll(m & ((1ull << lane) - 1ull));
      if (act[h]) {
        act_off[pos] = off[h];
        act_slot[pos] = (short)(tid + h * NT);
        act_rows[pos] = (char)nrow[h];
        act_cols[pos] = (char)ncol[h];
      }
      base += total;
      __syncthreads();
    }
    n_act = base;
  }

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
    zofs[k] = (r + ZR) * W3P + c + ZC;
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
  float sacc[SLOTS_PT];
  int s_off[SLOTS_PT], s_nr[SLOTS_PT], s_nc[SLOTS_PT];
  bool s_live[SLOTS_PT];
#pragma unroll
  for (int k = 0; k < SLOTS_PT; ++k) {
    const int m = min(lt + k * GT, NS - 1);
    sacc[k] = 0.0f;
    s_live[k] = lt + k * GT < n_act;
    s_off[k] = s_live[k] ? act_off[m] : 0;
    s_nr[k] = s_live[k] ? act_rows[m] : KS;
    s_nc[k] = s_live[k] ? act_cols[m] : KS;
  }

  __syncthreads();

  const int nf = pb.nf;
  for (int c0 = 0; c0 < nf; c0 += NC) {
    const int ncur = min(NC, nf - c0);
    for (int t = tid; t < KK * NC; t += NT) kf_s[t] = a.kf[(size_t)c0 * KK + t];
    for (int t = tid; t < NC * KAP; t += NT) {
      const int j = t / KAP, tt = t - j * KAP;
      ka_s[t] = tt < KK ? a.ka[(size_t)(c0 + j) * KK + tt] : 0.0f;
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
#pragma unroll
        for (int j = 0; j < NC; ++j) zp[j * PLANEP + zofs[k]] = zv[j];
      }
    } else if constexpr (FWD == FWD_MFMA_BF16) {
      // ---- stage 2 (matrix cores, BF16 operands, FP32 accumulation): v_mfma_f32_16x16x32_bf16 with
      // lane (m = lane % 16, k = lane / 16) holding taps 32s + 8k .. 32s + 8k + 7 of filter m (A) and the
      // same taps of position m (B).  The B values are differences u(p + t) - u(p) to the position's own
      // sample, so that BF16 rounding acts on local contrast and not on the 8-bit intensity level
      // (zero-sum filters applied to flat regions would otherwise drown in rounding noise); the exact
      // FP32 term u(p) * sum_t k[t] is added back after the product.  Each operand is split into a BF16
      // head and a BF16 tail (x = hi + lo), and three products hi*hi + hi*lo + lo*hi are accumulated,
      // which keeps the energies of the line search at close to FP32 accuracy.
      const int lane = tid & 63, wave = tid >> 6, lm = lane & 15, lk = lane >> 4;
      bf16x8 a16[2], a16lo[2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int t = 32 * s + 8 * lk + i;
          const float kv = t < KK ? kf_s[t * NC + lm] : 0.0f;
          a16[s][i] = (__bf16)kv;
          a16lo[s][i] = (__bf16)(kv - (float)a16[s][i]);
        }
      float thv[4], ksum[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int fj = 4 * lk + j;
        thv[j] = fj < ncur ? a.theta[c0 + fj] : 0.0f;
        float sum = 0.0f;
        for (int t = 0; t < KK; ++t) sum += kf_s[t * NC + fj];
        ksum[j] = sum;
      }
#pragma unroll 1
      for (int g = wave; g < NGROUP; g += NT / 64) {
        const int p = g * 16 + lm;
        const bool inr = p < PLANE3;
        const int r = inr ? p / W3 : 0, c = inr ? p - (p / W3) * W3 : 0;
        const int pbase = r * W6 + c;
        const float uc = u6[pbase + R * W6 + R];
        floatx4 acc4 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          bf16x8 b16, b16lo;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int t = 32 * s + 8 * lk + i;
            const int toff = t < KK ? (t / KS) * W6 + (t % KS) : 0;
            const float d = u6[pbase + toff] - uc;
            b16[i] = (__bf16)d;
            b16lo[i] = (__bf16)(d - (float)b16[i]);
          }
          acc4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a16lo[s], b16, acc4, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a16[s], b16lo, acc4, 0, 0, 0);
          acc4 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a16[s], b16, acc4, 0, 0, 0);
        }
        const int gy = y0 - R + r, gx = x0 - R + c;
        const bool inimg = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
        const bool live = inr && (inimg || bc == PERIODIC);
        const bool own = inr && inimg && r >= R && r < R + TH && c >= R && c < R + TW;
        const int zo = (r + ZR) * W3P + c + ZC;
        // the position's u(p) is the same for the 4 filters of this lane; fetch it per lane
        float e = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float yv = fmaf(uc, ksum[j], acc4[j]);
          const float den = fmaf(yv, yv, 1.0f);
          const float z = thv[j] * 2.0f * yv * fast_rcp(den);
          if (inr) zp[(4 * lk + j) * PLANEP + zo] = live ? z : 0.0f;
          if (UNF == FWD_HALF && own && 4 * lk + j < ncur)
            a.zbuf[(size_t)(c0 + 4 * lk + j) * a.zstride + im.off + (size_t)gy * W + gx] = z;
          e = fmaf(thv[j], fast_log(den), e);
        }
        if (own) accF += (double)e;
      }
    } else if constexpr (FWD == FWD_MFMA_F32) {
      // ---- stage 2 (matrix cores): per group of 16 consecutive R3 positions,
      // Y^T[16 filters x 16 positions] = Kflip^T[16 x 52 taps] . X[52 taps x 16 positions] with
      // v_mfma_f32_16x16x4f32 (taps 49..51 carry zero weight).  Lane (m = lane % 16, k = lane / 16)
      // holds the A value Kflip[filter m][tap 4s + k] and the B value u6 at tap 4s + k of position m;
      // the result lands as y for position m, filters 4k .. 4k + 3.
      const int lane = tid & 63, wave = tid >> 6, lm = lane & 15, lk = lane >> 4;
      float a_reg[13];
      int toff[13];
#pragma unroll
      for (int s = 0; s < 13; ++s) {
        const int t = 4 * s + lk;
        a_reg[s] = t < KK ? kf_s[t * NC + lm] : 0.0f;
        toff[s] = t < KK ? (t / KS) * W6 + (t % KS) : 0;
      }
      float thv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) thv[j] = 4 * lk + j < ncur ? a.theta[c0 + 4 * lk + j] : 0.0f;
      // two position groups per pass: two independent accumulator chains keep the matrix pipe busy
      // while each MFMA waits for its predecessor
#pragma unroll 1
      for (int g0 = wave; g0 < NGROUP; g0 += 2 * (NT / 64)) {
        int pb2[2], rr[2], cc[2];
        bool inr2[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int p = (g0 + h * (NT / 64)) * 16 + lm;
          inr2[h] = p < PLANE3;
          rr[h] = inr2[h] ? p / W3 : 0;
          cc[h] = inr2[h] ? p - rr[h] * W3 : 0;
          pb2[h] = rr[h] * W6 + cc[h];
        }
        floatx4 acc2[2] = {{0.0f, 0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int s = 0; s < 13; ++s)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            acc2[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_reg[s], u6[pb2[h] + toff[s]], acc2[h], 0, 0, 0);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = rr[h], c = cc[h];
          const bool inr = inr2[h];
          const int gy = y0 - R + r, gx = x0 - R + c;
          const bool inimg = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
          const bool live = inr && (inimg || bc == PERIODIC);
          const bool own = inr && inimg && r >= R && r < R + TH && c >= R && c < R + TW;
          const int zo = (r + ZR) * W3P + c + ZC;
          float e = 0.0f;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float yv = acc2[h][j];
            const float den = fmaf(yv, yv, 1.0f);
            const float z = thv[j] * 2.0f * yv * fast_rcp(den);
            if (inr) zp[(4 * lk + j) * PLANEP + zo] = live ? z : 0.0f;
            if (UNF == FWD_HALF && own && 4 * lk + j < ncur)
              a.zbuf[(size_t)(c0 + 4 * lk + j) * a.zstride + im.off + (size_t)gy * W + gx] = z;
            e = fmaf(thv[j], fast_log(den), e);
          }
          if (own) accF += (double)e;
        }
      }
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
          float th = j < ncur ? a.theta[c0 + j] : 0.0f;
          float den = fmaf(y[k][j], y[k][j], 1.0f);
          float z = th * 2.0f * y[k][j] * fast_rcp(den);
          zp[j * PLANEP + zofs[k]] = flive[k] ? z : 0.0f;
          if (UNF == FWD_HALF && fown[k] && j < ncur) {
            const int idx = tid + k * NT, r = idx / W3, c = idx - r * W3;
            a.zbuf[(size_t)(c0 + j) * a.zstride + im.off + (size_t)(y0 - R + r) * W + (x0 - R + c)] = z;
          }
          e = fmaf(th, fast_log(den), e);
        }
        if (fown[k]) accF += (double)e;
      }
    }
    __syncthreads();

    // ---- stage 3: adjoint bank.  Per filter of the group: the BR x BC block of this thread from a
    // (BR+6) x (BC+6) window in registers; then, on fold tiles, the fold slots assigned to this
    // thread (7x7 windows around extended samples, the same 49 taps).
#pragma unroll 1
    for (int jj = 0; jj < (UNF == FWD_HALF ? 0 : FPG); ++jj) {
      const int j = grp * FPG + jj;
      if (j >= ncur) break;
      float kt[KAP];
#pragma unroll
      for (int t = 0; t < KAP; t += 4) {
        float4 q4 = *reinterpret_cast<const float4*>(ka_s + j * KAP + t);
        kt[t] = q4.x; kt[t + 1] = q4.y; kt[t + 2] = q4.z; kt[t + 3] = q4.w;
      }
      const float* zplane = zp + j * PLANEP;
      const float* zb = zplane + (row0 + ZR) * W3P + col0 + ZC;
      // stream the (BR+6) x (BC+6) window one row at a time; row q feeds output rows q - ta
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        float wrow[WC];
#pragma unroll
        for (int s = 0; s < WC; s += 2) {
          float2 v2 = *reinterpret_cast<const float2*>(zb + q * W3P + s);
          wrow[s] = v2.x;
          wrow[s + 1] = v2.y;
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
    // the fold slots of this thread, filter by filter, in a pass of their own so that the window
    // loads of the regular blocks and of the slots do not compete for registers
    if (fold) {
#pragma unroll 1
      for (int jj = 0; jj < FPG; ++jj) {
        const int j = grp * FPG + jj;
        if (j >= ncur) break;
        float kt[KAP];
#pragma unroll
        for (int t = 0; t < KAP; t += 4) {
          float4 q4 = *reinterpret_cast<const float4*>(ka_s + j * KAP + t);
          kt[t] = q4.x; kt[t + 1] = q4.y; kt[t + 2] = q4.z; kt[t + 3] = q4.w;
        }
        const float* zplane = zp + j * PLANEP;
#pragma unroll
        for (int k = 0; k < SLOTS_PT; ++k) {
          if (!s_live[k]) break;
          const float* zw = zplane + s_off[k];
          // branch-free: every load is issued unconditionally.  Window rows 5, 6 and column 6 that
          // would leave the plane read the last in-plane row / column instead and are weighted zero
          // (row and column offsets and weights are arithmetic, so no load waits behind a branch).
          const int rofs5 = min(5, s_nr[k] - 1) * W3P, rofs6 = min(6, s_nr[k] - 1) * W3P;
          const int cofs6 = min(6, s_nc[k] - 1);
          const float m5 = (float)(s_nr[k] > 5), m6 = (float)(s_nr[k] > 6), mc6 = (float)(s_nc[k] > 6);
          float v = 0.0f;
#pragma unroll
          for (int ta = 0; ta < KS; ++ta) {
            const float* zr = zw + (ta < 5 ? ta * W3P : (ta == 5 ? rofs5 : rofs6));
            const float mr = ta < 5 ? 1.0f : (ta == 5 ? m5 : m6);
#pragma unroll
            for (int tb = 0; tb < KS; ++tb) {
              const float w = tb < 6 ? kt[ta * KS + tb] : kt[ta * KS + tb] * mc6;
              v = fmaf(ta < 5 ? w : w * mr, zr[tb < 6 ? tb : cofs6], v);
            }
          }
          sacc[k] += v;
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: combine groups and fold slots in a fixed order, chain rule, store
  if constexpr (UNF == FWD_HALF) {
    double v[5] = {accF, accG, accS1, accS2, accM};
    block_partials<NT, 5>(v, red, a.partials);
    return;
  }
  float* gsum = zp;                       // [NG][TH][TW]
  float* slots = zp + NG * TH * TW;       // [NG][NS]
#pragma unroll
  for (int i = 0; i < BR; ++i)
#pragma unroll
    for (int jx = 0; jx < BC; ++jx) gsum[grp * TH * TW + (row0 + i) * TW + col0 + jx] = acc[i][jx];
  if (fold) {
    for (int i = tid; i < NG * NS; i += NT) slots[i] = 0.0f;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SLOTS_PT; ++k) {
      const int m = lt + k * GT;
      if (m < n_act) slots[grp * NS + act_slot[m]] = sacc[k];
    }
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
      const int cb = 6 * TW + 6 * TH;
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const float* sl = slots + q * NS;
        if (py < R) g += sl[py * TW + jx];
        if (py >= H - R) g += sl[3 * TW + (H - 1 - py) * TW + jx];
        if (px < R) g += sl[6 * TW + px * TH + i];
        if (px >= W - R) g += sl[6 * TW + 3 * TH + (W - 1 - px) * TH + i];
        if (py < R && px < R) g += sl[cb + 0 * 9 + py * 3 + px];
        if (py < R && px >= W - R) g += sl[cb + 1 * 9 + py * 3 + (W - 1 - px)];
        if (py >= H - R && px < R) g += sl[cb + 2 * 9 + (H - 1 - py) * 3 + px];
        if (py >= H - R && px >= W - R) g += sl[cb + 3 * 9 + (H - 1 - py) * 3 + (W - 1 - px)];
      }
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
