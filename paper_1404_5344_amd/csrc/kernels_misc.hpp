// Small kernels of the iPiano loop: initial state, line-search decision, output, prox probe.
#pragma once
#include "device_math.hpp"

namespace foe {

// x^0 = x^{-1} = log u0 (log models) or u0 (IDIV), u0 = init or f.  Flags invalid input.
// Grid: (blocks, images); block row blockIdx.y covers image blockIdx.y.
__global__ void init_state_kernel(const float* __restrict__ f, const float* __restrict__ u0, float* x0, float* x1,
                                  const ImageDesc* images, int model, DevState* states) {
  const ImageDesc im = images[blockIdx.y];
  const size_t n = (size_t)im.off + (size_t)im.H * im.W;
  DevState* st = states + blockIdx.y;
  size_t i = (size_t)im.off + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float fv = f[i];
    float uv = u0 ? u0[i] : fv;
    bad |= !(fv > 0.0f && fv <= 3.0e38f) || !(uv > 0.0f && uv <= 3.0e38f);
    float x = model == IDIV ? uv : logf(uv);
    x0[i] = x;
    x1[i] = x;
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->input_bad, 1);
}

// Validity check of caller-provided state (resumable entry point).
__global__ void check_input_kernel(const float* __restrict__ f, const ImageDesc* images, DevState* states) {
  const ImageDesc im = images[blockIdx.y];
  const size_t n = (size_t)im.off + (size_t)im.H * im.W;
  DevState* st = states + blockIdx.y;
  size_t i = (size_t)im.off + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  for (; i < n; i += (size_t)gridDim.x * blockDim.x) {
    float fv = f[i];
    bad |= !(fv > 0.0f && fv <= 3.0e38f);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&st->input_bad, 1);
}

enum DecideMode { DECIDE_STEP = 0, DECIDE_INIT = 1, DECIDE_REPORT = 2 };

// Single-block reduction of the per-block partials in the fixed order of image_totals, then by mode: REPORT
// stores the totals; INIT also takes F(x^0) and checks the inputs; STEP settles a trial that has run and awaits
// its decision (decide_step).  One block per image (every thread of the block calls it: it contains a barrier).
__device__ __forceinline__ void decide_block(DevState* st, const double* __restrict__ partials, const ImageDesc& im,
                                             const Problem& pb, double* stats, int mode) {
  __shared__ double red[4 * 5];
  double tot[5];
  image_totals(partials, im.tile0, im.ntiles, red, tot);
  if (threadIdx.x != 0) return;
  DevState s = *st;
  if (mode == DECIDE_STEP) {
    if (!s.pending) return;   // nothing ran since the last decision
    s.pending = 0;
  }
  for (int k = 0; k < PART_COLS; ++k) s.sums[k] = k < 5 ? tot[k] : 0.0;
  if (mode == DECIDE_INIT) {
    s.t_start = (long long)wall_clock64();   // the iterations start now (per-image latency)
    s.t_done = 0;
    s.Fcur = tot[0];
    if (s.input_bad) {
      s.status = ST_EINPUT;
      s.done = 1;
    } else if (!isfinite(tot[0]) || !isfinite(tot[1])) {
      s.status = ST_ENONFINITE;
      s.done = 1;
    }
    if (s.target <= 0) s.done = 1;
  } else if (mode == DECIDE_STEP) {
    decide_step(s, tot, pb, stats);
  }
  *st = s;
}

// One block per image: block b reduces the partials of image b's tiles and decides.
__global__ __launch_bounds__(256) void decide_kernel(DevState* states, const double* __restrict__ partials,
                                                     const ImageDesc* images, Problem pb, double* stats_all,
                                                     int stats_rows, int mode) {
  DevState* st = states + blockIdx.x;
  if (mode == DECIDE_STEP && st->done) return;
  const ImageDesc im = images[blockIdx.x];
  decide_block(st, partials, im, pb, stats_all + (size_t)blockIdx.x * stats_rows * STAT_COLS, mode);
}

// u = e^{x^n} (log models) or x^n, from the ring slot each image's state names.
__global__ void finalize_kernel(const DevState* states, const float* x0, const float* x1, const float* x2, float* u,
                                const ImageDesc* images, int model) {
  const ImageDesc im = images[blockIdx.y];
  const size_t n = (size_t)im.off + (size_t)im.H * im.W;
  const float* x = pick3(states[blockIdx.y].icur, (float*)x0, (float*)x1, (float*)x2);
  for (size_t i = (size_t)im.off + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    u[i] = model == IDIV ? x[i] : expf(x[i]);
}

// Copy the ring slots the state names into caller buffers (resumable entry point).
__global__ void export_state_kernel(const DevState* states, const float* x0, const float* x1, const float* x2,
                                    float* xcur, float* xprev, const ImageDesc* images) {
  const ImageDesc im = images[blockIdx.y];
  const size_t n = (size_t)im.off + (size_t)im.H * im.W;
  const float* c = pick3(states[blockIdx.y].icur, (float*)x0, (float*)x1, (float*)x2);
  const float* p = pick3(states[blockIdx.y].iprev, (float*)x0, (float*)x1, (float*)x2);
  for (size_t i = (size_t)im.off + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    xcur[i] = c[i];
    xprev[i] = p[i];
  }
}

// The tile list of one image in row-major tile order (the order build_tiles gives on the host):
// tile t = (image 0, x0 = (t % ntx) tw, y0 = (t / ntx) th).
__global__ void tile_list_kernel(TileDesc* tiles, int ntx, int ntiles, int tw, int th) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ntiles; i += gridDim.x * blockDim.x) {
    const int t = xcd_tile_order(i, ntiles);
    tiles[i] = TileDesc{0, (t % ntx) * tw, (t / ntx) * th, 0};
  }
}

__global__ void prox_probe_kernel(const float* __restrict__ xh, const float* __restrict__ f, float* out, size_t n,
                                  float tau, Problem pb, float lam1, float lam2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = prox_pixel(xh[i], f[i], tau, pb.model, lam1, lam2, pb.newton_iters, pb.prox_method);
}

}  // namespace foe
