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

struct FusedArgs {
  Problem pb;
  const float* f;
  float* xr0; float* xr1; float* xr2;   // x ring (TRIAL)
  float* gr0; float* gr1;               // gradient ring (TRIAL)
  const float* x_in;                    // EVAL input
  float* g_out;                         // EVAL output
  DevState* st;
  double* partials;                     // [gridDim.x][PART_COLS]
  const float* kf;                      // forward taps, flipped and chunk-transposed:
                                        //   kf[(c * KK + a * 7 + b) * NC + j] = k_{c*NC+j}[6-a][6-b]
  const float* ka;                      // adjoint taps: ka[i][a][b] = k_i[a][b]
  const float* theta;
  int tiles_x;
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

// Fold slots of the SYMMETRIC boundary map: the extended samples q != p with source p.
// Slot layout (TW/TH = tile width/height):
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

template <int TW, int TH, int NC, int NT, int NG>
__global__ __launch_bounds__(NT) void fused_valu_kernel(FusedArgs a) {
  constexpr int W6 = TW + 4 * R, H6 = TH + 4 * R;
  constexpr int W3 = TW + 2 * R, H3 = TH + 2 * R;
  constexpr int PLANE3 = H3 * W3;
  constexpr int GT = NT / NG;              // threads per adjoint group
  constexpr int FPG = NC / NG;             // filters per group per chunk
  constexpr int STRIPS = GT / TW;          // strips per column
  constexpr int STRIP = TH / STRIPS;       // rows per thread
  constexpr int NS = 6 * TW + 6 * TH + 36; // fold slots
  constexpr int SLOTS_PT = (NS + NT - 1) / NT;
  static_assert(GT % TW == 0 && TH % STRIPS == 0 && NC % NG == 0 && GT % 64 == 0, "bad tiling");
  static_assert(NG * TH * TW + NS <= NC * PLANE3, "epilogue does not fit in the z buffer");

  __shared__ float u6[H6 * W6];
  __shared__ float z3[NC * PLANE3];
  __shared__ double red[(NT / 64) * 5];

  const int tid = threadIdx.x;
  const Problem pb = a.pb;
  const int H = pb.H, W = pb.W, bc = pb.bc, model = pb.model;
  const bool logm = model != IDIV;

  const float* xc;
  const float* xp = nullptr;
  const float* gc = nullptr;
  float* xo = nullptr;
  float* go;
  float alpha = 0.0f;
  if (a.mode == MODE_TRIAL) {
    const DevState* st = a.st;
    if (st->done) return;
    alpha = (float)st->alpha;
    xc = pick3(st->icur, a.xr0, a.xr1, a.xr2);
    xp = pick3(st->iprev, a.xr0, a.xr1, a.xr2);
    xo = pick3(st->icand, a.xr0, a.xr1, a.xr2);
    gc = pick2(st->gcur, a.gr0, a.gr1);
    go = pick2(st->gcand, a.gr0, a.gr1);
  } else {
    xc = a.x_in;
    go = a.g_out;
  }
  const float* __restrict__ f = a.f;

  const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
  const int x0 = tx * TW, y0 = ty * TH;

  double accF = 0.0, accG = 0.0, accS1 = 0.0, accS2 = 0.0, accM = 0.0;

  // ---- stage 1: step + prox on tile + 6 halo -> u6
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
        xn = prox_pixel(xh, fv, alpha, model, pb.lam1, pb.lam2, pb.newton_iters);
        uval = logm ? fast_exp(xn) : xn;
        if (own) {
          xo[p] = xn;
          float d = xn - xv, m = xv - xpv;
          accS1 += (double)(gv * d);
          accS2 += (double)(d * d);
          accM += (double)(m * m);
          accG += (double)data_term(xn, uval, fv, model, pb.lam1, pb.lam2);
        }
      } else {
        xn = xc[p];
        uval = logm ? fast_exp(xn) : xn;
        if (own) accG += (double)data_term(xn, uval, fv, model, pb.lam1, pb.lam2);
      }
    }
    u6[idx] = uval;
  }
  __syncthreads();

  // ---- adjoint mapping
  const int grp = __builtin_amdgcn_readfirstlane(tid / GT);  // wave-uniform (GT % 64 == 0)
  const int lt = tid - grp * GT;
  const int col = lt % TW;
  const int row0 = (lt / TW) * STRIP;
  float acc[STRIP];
#pragma unroll
  for (int k = 0; k < STRIP; ++k) acc[k] = 0.0f;

  const bool fold = bc == SYMMETRIC && (y0 < R || y0 + TH > H - R || x0 < R || x0 + TW > W - R);
  float sacc[SLOTS_PT];
#pragma unroll
  for (int k = 0; k < SLOTS_PT; ++k) sacc[k] = 0.0f;

  const int nf = pb.nf;
  for (int c0 = 0; c0 < nf; c0 += NC) {
    const int ncur = min(NC, nf - c0);
    // ---- stage 2: forward bank + rho, rho' on tile + 3 halo -> z3
    for (int idx = tid; idx < PLANE3; idx += NT) {
      int r = idx / W3, c = idx - r * W3;
      int gy = y0 - R + r, gx = x0 - R + c;
      bool inimg = (unsigned)gy < (unsigned)H && (unsigned)gx < (unsigned)W;
      if (!inimg && bc != PERIODIC) {
#pragma unroll
        for (int j = 0; j < NC; ++j) z3[j * PLANE3 + idx] = 0.0f;
        continue;
      }
      float y[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) y[j] = 0.0f;
      cfloat* kb = as_const(a.kf) + (size_t)c0 * KK;   // chunk c0 / NC, [t][j]
      // one filter row at a time keeps 7 x NC taps in SGPRs
#pragma unroll 1
      for (int ta = 0; ta < KS; ++ta) {
        float wrow[KS];
#pragma unroll
        for (int tb = 0; tb < KS; ++tb) wrow[tb] = u6[(r + ta) * W6 + c + tb];
        cfloat* kr = kb + ta * KS * NC;
#pragma unroll
        for (int tb = 0; tb < KS; ++tb)
#pragma unroll
          for (int j = 0; j < NC; ++j) y[j] = fmaf(kr[tb * NC + j], wrow[tb], y[j]);
      }
      const bool own = inimg && r >= R && r < R + TH && c >= R && c < R + TW;
      float e = 0.0f;
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        float th = j < ncur ? as_const(a.theta)[c0 + j] : 0.0f;
        float den = fmaf(y[j], y[j], 1.0f);
        z3[j * PLANE3 + idx] = th * 2.0f * y[j] * fast_rcp(den);
        e = fmaf(th, fast_log(den), e);
      }
      if (own) accF += (double)e;
    }
    __syncthreads();

    // ---- stage 3: adjoint bank on the tile (strips of STRIP rows), group grp takes FPG filters
#pragma unroll 1
    for (int jj = 0; jj < FPG; ++jj) {
      const int j = grp * FPG + jj;
      if (j >= ncur) break;
      cfloat* kj = as_const(a.ka) + (size_t)(c0 + j) * KK;
      const float* zb = z3 + j * PLANE3;
#pragma unroll
      for (int tb = 0; tb < KS; ++tb) {
        float colv[STRIP + KS - 1];
#pragma unroll
        for (int q = 0; q < STRIP + KS - 1; ++q) colv[q] = zb[(row0 + q) * W3 + col + tb];
#pragma unroll
        for (int ta = 0; ta < KS; ++ta) {
          const float kv = kj[ta * KS + tb];
#pragma unroll
          for (int k = 0; k < STRIP; ++k) acc[k] = fmaf(kv, colv[k + ta], acc[k]);
        }
      }
    }
    // mirror terms of the SYMMETRIC map: v(q) = sum_j sum_ab k_j[a][b] z_j(q + (a-3, b-3)), z = 0 off the image
    if (fold) {
#pragma unroll
      for (int k = 0; k < SLOTS_PT; ++k) {
        int s = tid + k * NT;
        int ply, plx, qy, qx;
        if (s < NS && slot_target<TW, TH>(s, x0, y0, H, W, ply, plx, qy, qx)) {
          float v = 0.0f;
          for (int j = 0; j < ncur; ++j) {
            cfloat* kj = as_const(a.ka) + (size_t)(c0 + j) * KK;
            const float* zb = z3 + j * PLANE3;
            for (int ta = 0; ta < KS; ++ta) {
              int zy = qy - R + ta;
              if ((unsigned)zy >= (unsigned)H) continue;
              int r3 = zy - (y0 - R);
              if ((unsigned)r3 >= (unsigned)H3) continue;
              for (int tb = 0; tb < KS; ++tb) {
                int zx = qx - R + tb;
                if ((unsigned)zx >= (unsigned)W) continue;
                int c3 = zx - (x0 - R);
                if ((unsigned)c3 >= (unsigned)W3) continue;
                v = fmaf(kj[ta * KS + tb], zb[r3 * W3 + c3], v);
              }
            }
          }
          sacc[k] += v;
        }
      }
    }
    __syncthreads();
  }

  // ---- epilogue: combine groups and fold slots in a fixed order, chain rule, store
  float* gsum = z3;                       // [NG][TH][TW]
  float* slots = z3 + NG * TH * TW;       // [NS]
#pragma unroll
  for (int k = 0; k < STRIP; ++k) gsum[grp * TH * TW + (row0 + k) * TW + col] = acc[k];
  if (fold) {
#pragma unroll
    for (int k = 0; k < SLOTS_PT; ++k) {
      int s = tid + k * NT;
      if (s < NS) slots[s] = sacc[k];
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
      if (py < R) g += slots[py * TW + jx];
      if (py >= H - R) g += slots[3 * TW + (H - 1 - py) * TW + jx];
      if (px < R) g += slots[6 * TW + px * TH + i];
      if (px >= W - R) g += slots[6 * TW + 3 * TH + (W - 1 - px) * TH + i];
      const int cb = 6 * TW + 6 * TH;
      if (py < R && px < R) g += slots[cb + 0 * 9 + py * 3 + px];
      if (py < R && px >= W - R) g += slots[cb + 1 * 9 + py * 3 + (W - 1 - px)];
      if (py >= H - R && px < R) g += slots[cb + 2 * 9 + (H - 1 - py) * 3 + px];
      if (py >= H - R && px >= W - R) g += slots[cb + 3 * 9 + (H - 1 - py) * 3 + (W - 1 - px)];
    }
    if (logm) g *= u6[(i + 2 * R) * W6 + jx + 2 * R];
    go[(size_t)py * W + px] = g;
  }

  double v[5] = {accF, accG, accS1, accS2, accM};
  block_partials<NT, 5>(v, red, a.partials);
}

}  // namespace foe
