// Pointwise device functions of the FoE + iPiano path: boundary map, data terms, prox.
#pragma once
#include "common.hpp"

namespace foe {

// The backtracking decision on a trial (iPiano, as Sec. II-C adopts it) from the totals of its block
// partials tot = {F(x+), G(x+), <grad F(x), d>, |d|^2, |x - x_prev|^2}, applied to a copy s of the
// image's state: accept iff F(x+) <= F(x) + <grad F(x), d> + L/2 |d|^2 (descent lemma), which a
// non-finite F(x+) or G(x+) fails; on acceptance rotate the x and gradient rings and write the stats row
// (row: the image's stats, or null to skip the write); on rejection L <- eta_up L.  FIXED mode always
// accepts.
__device__ __forceinline__ void decide_step_core(DevState& s, const double (&tot)[5], const Problem& pb, double* row) {
  const double F = tot[0], G = tot[1], s1 = tot[2], s2 = tot[3], m = tot[4];
  s.trials += 1;
  s.total_trials += 1;
  const bool finite = isfinite(F) && isfinite(G) && isfinite(s1) && isfinite(s2);
  if (!finite && pb.step_mode == FIXED) {
    s.status = ST_ENONFINITE;
    s.done = 1;
    return;
  }
  const double L = s.L;
  // a trial with a non-finite energy fails the descent test and is rejected like any other
  const bool accept = finite && (pb.step_mode == FIXED || F <= s.Fcur + s1 + 0.5 * L * s2);
  if (accept) {
    if (row) {
      row += (size_t)s.iter * STAT_COLS;
      row[0] = F; row[1] = G; row[2] = L; row[3] = s.alpha;
      row[4] = (double)s.trials; row[5] = s1; row[6] = s2; row[7] = m;
    }
    const int c = s.icur, p = s.iprev, n = s.icand;
    s.icur = n; s.iprev = c; s.icand = p;
    const int g = s.gcur;
    s.gcur = s.gcand; s.gcand = g;
    s.Fcur = F;
    s.L_acc = L;
    s.iter += 1;
    s.trials = 0;
    if (s.iter >= s.target) s.done = 1;
    if (pb.step_mode == BACKTRACK) {
      s.L = pb.eta_down * L;
      s.alpha = 1.9 * (1.0 - pb.beta_d) / s.L;
    }
  } else if (s.trials > pb.max_backtracks) {
    s.status = ST_ELINESEARCH;
    s.done = 1;
  } else {
    s.L = pb.eta_up * L;
    s.alpha = 1.9 * (1.0 - pb.beta_d) / s.L;
  }
}

// The decision, with the device wall-clock time at which it completes the image (per-image latency).
__device__ __forceinline__ void decide_step(DevState& s, const double (&tot)[5], const Problem& pb, double* row) {
  const int was_done = s.done;
  decide_step_core(s, tot, pb, row);
  if (s.done && !was_done) s.t_done = (long long)wall_clock64();
}

// One step of wave_sum_f64: v + (v moved by the DPP pattern CTRL; 0 where the pattern has no source
// or ROW_MASK leaves the row out).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of x over the 64 lanes of a wave, left in lane 63 (the other lanes hold partial sums): an
// inclusive scan with DPP moves, row shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the
// broadcasts of lane 15 of each row into the next row and of lane 31 into rows 2 and 3.  Register
// moves only (no LDS crossbar); the order of the additions is fixed.
__device__ __forceinline__ double wave_sum_f64(double x) {
  x = dpp_add_f64<0x111, 0xf>(x);   // row_shr:1
  x = dpp_add_f64<0x112, 0xf>(x);   // row_shr:2
  x = dpp_add_f64<0x114, 0xf>(x);   // row_shr:4
  x = dpp_add_f64<0x118, 0xf>(x);   // row_shr:8
  x = dpp_add_f64<0x142, 0xa>(x);   // row_bcast:15 -> rows 1, 3
  x = dpp_add_f64<0x143, 0xc>(x);   // row_bcast:31 -> rows 2, 3
  return x;
}

// Fixed-order FP64 totals of the five partial columns {F, G, s1, s2, m} of one image's tiles, shared by every
// kernel that decides on a trial (so that all of them round the same way): threads 0..255 of the block take
// tiles tile0 + t, t + 256, ... in that order, the four wave sums go through red (4 x 5 doubles, shared), and
// thread 0 receives tot[k] = ((w0 + w1) + w2) + w3.  Every thread of the block calls it (it holds a barrier).
__device__ __forceinline__ void image_totals(const double* __restrict__ part, int tile0, int ntiles, double* red,
                                             double (&tot)[5]) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (threadIdx.x < 256)
    for (int b = tile0 + (int)threadIdx.x; b < tile0 + ntiles; b += 256)
#pragma unroll
      for (int k = 0; k < 5; ++k) v[k] += part[(size_t)b * PART_COLS + k];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double x = wave_sum_f64(v[k]);
    if (lane == 63 && wave < 4) red[wave * 5 + k] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) tot[k] = red[k] + red[5 + k] + red[10 + k] + red[15 + k];
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// e^x through the hardware 2^x
__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
// ln x through the hardware log2
__device__ __forceinline__ float fast_log(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }

// Read-only data addressed through the constant address space: wave-uniform loads from it
// become scalar loads (filter taps and weights live in SGPRs, not VGPRs).
typedef const __attribute__((address_space(4))) float cfloat;
__device__ __forceinline__ cfloat* as_const(const float* p) { return (cfloat*)p; }

// Ring-buffer selection by a state index without indexing the kernel-argument block.
__device__ __forceinline__ float* pick3(int i, float* a, float* b, float* c) { return i == 0 ? a : (i == 1 ? b : c); }
__device__ __forceinline__ float* pick2(int i, float* a, float* b) { return i == 0 ? a : b; }

// Boundary map of the 3-pixel extension: extended index q -> source pixel, or -1 where the
// extension is zero or the sample is never read (SYMMETRIC beyond 3 pixels).
__device__ __forceinline__ int bmap(int q, int n, int bc) {
  if ((unsigned)q < (unsigned)n) return q;
  if (bc == PERIODIC) {
    int r = q % n;
    return r < 0 ? r + n : r;
  }
  if (bc == SYMMETRIC && q >= -R && q < n + R) return q < 0 ? -1 - q : 2 * n - 1 - q;
  return -1;
}

// Per-pixel data term G_p(x; f) of the three models; u = e^x for the log models, u = x for IDIV.
__device__ __forceinline__ float data_term(float x, float u, float f, int model, float lam1, float lam2) {
  float f2 = f * f;
  if (model == IDIV) return 0.5f * lam1 * (x * x - 2.0f * f2 * fast_log(x));
  float iu = fast_rcp(u);
  float t = 0.5f * lam1 * (2.0f * x + f2 * iu * iu);
  if (model == COMBINED) t += 0.5f * lam2 * (u * u - 2.0f * f2 * x);
  return t;
}

// prox_{tau G}(xh) at one pixel.
// Log models: the root of phi(w) = w - xh + tau lam1 (1 - f^2 e^{-2w}) + tau lam2 (e^{2w} - f^2),
// solved for t = w - log f (so f^2 e^{-2w} = e^{-2t}): Newton's method from t = xh - log f, kept
// inside the bracket [min(t_hat, 0), max(t_hat, 0)] that holds the root (both data terms are
// minimised at w = log f, and phi is increasing); a step that leaves the bracket or is not
// finite is replaced by bisection.  Each pixel stops at |dt| <= 4e-7 max(1, |w|) or after
// max_iters iterations; the loop ends when every pixel of the wavefront has stopped.  A
// pixel's result depends only on its own inputs.
// IDIV: the positive root of (1 + tau lam) u^2 - xh u - tau lam f^2 = 0, in the form
// without cancellation for xh < 0.
// LOG model, direct solve (Sec. II-C names the Lambert W route).  In t = w - log f the prox minimises
// (t - t_hat)^2 / 2 + a (t + e^{-2t} / 2), a = tau lam1, whose optimality condition
// t - t_hat + a (1 - e^{-2t}) = 0 has the solution t = t_hat - a + y / 2, y = W0(z), z = 2 a e^{2 (a - t_hat)}
// (W0 = principal branch of Lambert's W).  Since y + ln y = ln z, this equals t = (ln 2a - ln y) / 2, which
// has no cancellation when a and y / 2 are both large.  y is taken from ln z (no overflow for large z) by
// three Newton steps on y + ln y = ln z, started from ln z - ln ln z (ln z > 1) or z / (1 + z); for
// ln z < -60, ln y = ln z to FP32 accuracy.
__device__ __forceinline__ float prox_log_lambertw(float xh, float f, float tau, float lam1) {
  const float a = tau * lam1;
  if (!(a > 0.0f)) return xh;
  const float lf = fast_log(f);
  const float l2a = fast_log(2.0f * a);
  const float lnz = l2a + 2.0f * (a - (xh - lf));
  float lny = lnz;
  if (lnz > -60.0f) {
    float y;
    if (lnz > 1.0f) {
      y = lnz - fast_log(lnz);
    } else {
      const float z = fast_exp(lnz);
      y = z * fast_rcp(1.0f + z);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) y = y * (1.0f + lnz - fast_log(y)) * fast_rcp(1.0f + y);
    lny = fast_log(y);
  }
  return 0.5f * (l2a - lny) + lf;
}

__device__ __forceinline__ float prox_pixel(float xh, float f, float tau, int model, float lam1, float lam2,
                                            int max_iters, int method = 0) {
  if (method == 1) return prox_log_lambertw(xh, f, tau, lam1);
  if (model == IDIV) {
    float a = 1.0f + tau * lam1;
    float c = tau * lam1 * f * f;
    float s = sqrtf(xh * xh + 4.0f * a * c);
    return xh >= 0.0f ? (xh + s) * fast_rcp(2.0f * a) : 2.0f * c * fast_rcp(s - xh);
  }
  const float a1 = tau * lam1;
  const float b2 = (model == COMBINED) ? tau * lam2 * f * f : 0.0f;
  const float lf = fast_log(f);
  const float th = xh - lf;
  float lo = fminf(th, 0.0f), hi = fmaxf(th, 0.0f);
  float t = th;
  bool done = false;
  for (int it = 0; it < max_iters; ++it) {
    if (!done) {
      float e = fast_exp(2.0f * t);          // e^{2t}
      float em = fast_rcp(e);                // e^{-2t}
      float phi = (t - th) + a1 * (1.0f - em) + b2 * (e - 1.0f);
      float dphi = 1.0f + 2.0f * a1 * em + 2.0f * b2 * e;
      if (phi > 0.0f) hi = fminf(hi, t); else if (phi < 0.0f) lo = fmaxf(lo, t);
      float tn = t - phi * fast_rcp(dphi);
      if (!(tn >= lo && tn <= hi)) tn = 0.5f * (lo + hi);
      done = fabsf(tn - t) <= 4e-7f * fmaxf(1.0f, fabsf(tn + lf)) || phi == 0.0f;
      t = tn;
    }
    if (__all(done)) break;
  }
  return t + lf;
}

}  // namespace foe
