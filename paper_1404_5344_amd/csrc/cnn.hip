// Warm-start network: six 3x3 convolutions (1 -> 32, 4 x 32 -> 32, 32 -> 1), zero "same"
// padding, ReLU after the first five, input log f - 4.5, output w0 = log f + net.  Hand-written
// forward, backward-data, backward-weight, loss and Adam kernels.  Weights are BF16 (the
// FP32 master weights rounded to BF16 after every Adam step); activations and accumulation
// are FP32.  Activations are NCHW planes.
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

// out[n][co][p] = act(bias[co] + sum_ci sum_t wt[ci][t][co] in[n][ci][p + off_t]) * (mask[n][co][p] > 0),
// act = ReLU when relu != 0; bias and mask nullable; zero padding.  wt is uniform across the
// block and is read through the scalar path.
template <int CI, int CO, int CICH>
__global__ __launch_bounds__(256) void conv3_kernel(const float* __restrict__ in, const float* __restrict__ wt,
                                                    const float* __restrict__ bias, float* __restrict__ out,
                                                    const float* __restrict__ mask, int H, int W, int relu) {
  __shared__ float tile[CICH][TS + 2][TS + 2];
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS, n = blockIdx.z;
  const size_t plane = (size_t)H * W;
  const float* inb = in + (size_t)n * CI * plane;
  foe::cfloat* w = foe::as_const(wt);
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias ? bias[co] : 0.0f;
  for (int c0 = 0; c0 < CI; c0 += CICH) {
    for (int i = threadIdx.x; i < CICH * (TS + 2) * (TS + 2); i += 256) {
      const int ci = i / ((TS + 2) * (TS + 2)), r = (i / (TS + 2)) % (TS + 2), c = i % (TS + 2);
      const int y = y0 + r - 1, x = x0 + c - 1;
      tile[ci][r][c] = (y >= 0 && y < H && x >= 0 && x < W) ? inb[(c0 + ci) * plane + (size_t)y * W + x] : 0.0f;
    }
    __syncthreads();
#pragma unroll 1
    for (int ci = 0; ci < CICH; ++ci)
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const float v = tile[ci][ty + t / 3][tx + t % 3];
        foe::cfloat* wr = w + ((size_t)(c0 + ci) * 9 + t) * CO;
#pragma unroll
        for (int co = 0; co < CO; ++co) acc[co] = fmaf(wr[co], v, acc[co]);
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

// Weight gradient of a 32 -> 32 layer, partial over a range of tiles:
//   dW[co][ci][t] += sum_p dout[co][p] in[ci][p + off_t],  db[co] += sum_p dout[co][p].
// Thread (co block of 4, ci block of 4, row group of 4) slides a 3x3 window along each row, so
// each step loads 3 new input samples per channel for 144 FMAs.  Grid: (tile groups, images).
// partial: [gridDim.y][gridDim.x][COUT*CIN*9 + COUT].
__global__ __launch_bounds__(256) void wgrad32_kernel(const float* __restrict__ in, const float* __restrict__ dout,
                                                      float* __restrict__ partial, int H, int W, int tiles_per_block) {
  constexpr int C = 32, NP = C * C * 9 + C;
  __shared__ float sin_[C][TS + 2][TS + 2];
  __shared__ float sd[C][TS][TS];
  __shared__ float red[4][C];
  __shared__ float gsum[4][C * C];
  const int cb = threadIdx.x & 7, ib = (threadIdx.x >> 3) & 7, pg = threadIdx.x >> 6;  // pg: wave-uniform
  const int n = blockIdx.y;
  const size_t plane = (size_t)H * W;
  const int tiles_x = (W + TS - 1) / TS, tiles_y = (H + TS - 1) / TS, ntiles = tiles_x * tiles_y;
  float acc[4][4][9];
  float bacc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    bacc[a] = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int t = 0; t < 9; ++t) acc[a][b][t] = 0.0f;
  }
  const float* inb = in + (size_t)n * C * plane;
  const float* db = dout + (size_t)n * C * plane;
  for (int tt = 0; tt < tiles_per_block; ++tt) {
    const int tile = blockIdx.x * tiles_per_block + tt;
    if (tile >= ntiles) break;
    const int x0 = (tile % tiles_x) * TS, y0 = (tile / tiles_x) * TS;
    for (int i = threadIdx.x; i < C * (TS + 2) * (TS + 2); i += 256) {
      const int ci = i / ((TS + 2) * (TS + 2)), r = (i / (TS + 2)) % (TS + 2), c = i % (TS + 2);
      const int y = y0 + r - 1, x = x0 + c - 1;
      sin_[ci][r][c] = (y >= 0 && y < H && x >= 0 && x < W) ? inb[ci * plane + (size_t)y * W + x] : 0.0f;
    }
    for (int i = threadIdx.x; i < C * TS * TS; i += 256) {
      const int co = i / (TS * TS), r = (i / TS) % TS, c = i % TS;
      const int y = y0 + r, x = x0 + c;
      sd[co][r][c] = (y < H && x < W) ? db[co * plane + (size_t)y * W + x] : 0.0f;
    }
    __syncthreads();
#pragma unroll 1
    for (int rr = 0; rr < 4; ++rr) {
      const int r = pg * 4 + rr;
      float win[4][3][3];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          win[b][dy][0] = 0.0f;
          win[b][dy][1] = sin_[ib * 4 + b][r + dy][0];
          win[b][dy][2] = sin_[ib * 4 + b][r + dy][1];
        }
#pragma unroll 2
      for (int c = 0; c < TS; ++c) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            win[b][dy][0] = win[b][dy][1];
            win[b][dy][1] = win[b][dy][2];
            win[b][dy][2] = sin_[ib * 4 + b][r + dy][c + 2];
          }
        float dv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) dv[a] = sd[cb * 4 + a][r][c];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          bacc[a] += dv[a];
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[a][b][t] = fmaf(dv[a], win[b][t / 3][t % 3], acc[a][b][t]);
        }
      }
    }
    __syncthreads();
  }
  // sum the 4 row groups in a fixed order through LDS, one tap at a time
  float* pout = partial + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NP;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) gsum[pg][(cb * 4 + a) * C + ib * 4 + b] = acc[a][b][t];
    __syncthreads();
    for (int i = threadIdx.x; i < C * C; i += 256) {
      const float s = ((gsum[0][i] + gsum[1][i]) + gsum[2][i]) + gsum[3][i];
      const int co = i / C, ci = i % C;
      pout[(co * C + ci) * 9 + t] = s;
    }
    __syncthreads();
  }
  if (ib == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a) red[pg][cb * 4 + a] = bacc[a];
  }
  __syncthreads();
  if (threadIdx.x < C) pout[C * C * 9 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
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
  for (int b = 0; b < nb; ++b) s += partial[(size_t)b * np + i];
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
  if (c->lpart) (void)hipFree(c->lpart);
  delete c;
}

constexpr int WG_TILES = 4;  // tiles per block of the 32 -> 32 weight-gradient kernel

int wgrad_groups(int H, int W) {
  const int tiles = ((W + TS - 1) / TS) * ((H + TS - 1) / TS);
  return (tiles + WG_TILES - 1) / WG_TILES;
}

foe_status reserve(foe_cnn* c, int n_img, int H, int W) {
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
  const size_t need = (size_t)n_img * wgrad_groups(H, W) * 9248;
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
  return FOE_OK;
}

void launch_conv(foe_cnn* c, int l, bool backward, const float* in, float* out, const float* mask, int n, int H,
                 int W) {
  dim3 grid((W + TS - 1) / TS, (H + TS - 1) / TS, n);
  const float* wf = c->wfwd + c->woffs[l];
  const float* wb = c->wbwd + c->woffs[l];
  const float* b = c->bias + c->boffs[l];
  if (!backward) {
    const int relu = l < NL - 1;
    if (l == 0)
      conv3_kernel<1, 32, 1><<<grid, 256, 0, c->stream>>>(in, wf, b, out, nullptr, H, W, relu);
    else if (l == NL - 1)
      conv3_kernel<32, 1, 8><<<grid, 256, 0, c->stream>>>(in, wf, b, out, nullptr, H, W, relu);
    else
      conv3_kernel<32, 32, 8><<<grid, 256, 0, c->stream>>>(in, wf, b, out, nullptr, H, W, relu);
  } else {
    // d_in = conv(d_out, flipped transposed taps) * (a_in > 0); the layer's input channels are the outputs
    if (l == NL - 1)
      conv3_kernel<1, 32, 1><<<grid, 256, 0, c->stream>>>(in, wb, nullptr, out, mask, H, W, 0);
    else
      conv3_kernel<32, 32, 8><<<grid, 256, 0, c->stream>>>(in, wb, nullptr, out, mask, H, W, 0);
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
  const int groups = wgrad_groups(H, W);
  for (int l = NL - 1; l >= 0; --l) {
    const int np = layer_params(l);
    float* g = c->grad + c->offs[l];
    if (CIN[l] == 32 && COUT[l] == 32) {
      wgrad32_kernel<<<dim3(groups, n), 256, 0, c->stream>>>(c->act[l], dcur, c->partial, H, W, WG_TILES);
      reduce_partials_kernel<<<(np + 255) / 256, 256, 0, c->stream>>>(c->partial, groups * n, np, g);
    } else if (l == 0) {
      wgrad_small_kernel<1, 32><<<dim3(groups, n), 256, 0, c->stream>>>(c->act[0], dcur, c->partial, H, W, WG_TILES);
      reduce_partials_kernel<<<(np + 255) / 256, 256, 0, c->stream>>>(c->partial, groups * n, np, g);
    } else {
      wgrad_small_kernel<32, 1><<<dim3(groups, n), 256, 0, c->stream>>>(c->act[l], dcur, c->partial, H, W, WG_TILES);
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
