// Image-quality index on the GPU: SSIM of an output against a reference image (Wang, Bovik, Sheikh
// and Simoncelli; the index the paper reports beside PSNR in Sec. III-B).  11 x 11 Gaussian window
// (standard deviation 1.5, normalised), C1 = (0.01 peak)^2, C2 = (0.03 peak)^2, mean of the SSIM map
// over the positions where the window lies inside the image.
//
// One workgroup per 32 x 16 block of window positions: the two images on the block + 10 halo are staged
// in LDS, a horizontal 11-tap pass forms the five weighted sums (x, y, x^2, y^2, x y) per row, a vertical
// pass finishes them per position; FP32 window sums, FP64 block sums reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/foe.h"

void foe_internal_set_error(const std::string& msg);

namespace quality {

constexpr int WIN = 11, TX = 32, TY = 16, NT = 256;
constexpr int IX = TX + WIN - 1, IY = TY + WIN - 1;

struct Taps {
  float w[WIN];
};

__global__ __launch_bounds__(NT) void ssim_blocks(const float* __restrict__ u, const float* __restrict__ ref, int H,
                                                  int W, Taps g, float c1, float c2, double* __restrict__ partial) {
  __shared__ float sx[IY][IX], sy[IY][IX];
  __shared__ float hp[5][IY][TX];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int ox = blockIdx.x * TX, oy = blockIdx.y * TY;  // first window position (its top-left pixel)
  const int Wo = W - WIN + 1, Ho = H - WIN + 1;
  for (int i = tid; i < IY * IX; i += NT) {
    const int r = i / IX, c = i - r * IX, y = oy + r, x = ox + c;
    const bool in = y < H && x < W;
    sx[r][c] = in ? u[(size_t)y * W + x] : 0.0f;
    sy[r][c] = in ? ref[(size_t)y * W + x] : 0.0f;
  }
  __syncthreads();
  for (int i = tid; i < IY * TX; i += NT) {
    const int r = i / TX, c = i - r * TX;
    float a = 0.f, b = 0.f, aa = 0.f, bb = 0.f, ab = 0.f;
#pragma unroll
    for (int t = 0; t < WIN; ++t) {
      const float xv = sx[r][c + t], yv = sy[r][c + t], wv = g.w[t];
      a = fmaf(wv, xv, a);
      b = fmaf(wv, yv, b);
      aa = fmaf(wv, xv * xv, aa);
      bb = fmaf(wv, yv * yv, bb);
      ab = fmaf(wv, xv * yv, ab);
    }
    hp[0][r][c] = a; hp[1][r][c] = b; hp[2][r][c] = aa; hp[3][r][c] = bb; hp[4][r][c] = ab;
  }
  __syncthreads();
  double acc = 0.0;
  for (int i = tid; i < TY * TX; i += NT) {
    const int r = i / TX, c = i - r * TX;
    if (oy + r >= Ho || ox + c >= Wo) continue;
    float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < WIN; ++t)
#pragma unroll
      for (int k = 0; k < 5; ++k) m[k] = fmaf(g.w[t], hp[k][r + t][c], m[k]);
    const float mx = m[0], my = m[1];
    const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const float num = (2.0f * mx * my + c1) * (2.0f * cxy + c2);
    const float den = (mx * mx + my * my + c1) * (vx + vy + c2);
    acc += (double)(num / den);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    partial[blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// out = sum of partial[0 .. n) / count, in a fixed order.
__global__ __launch_bounds__(NT) void ssim_total(const double* __restrict__ partial, int n, double count,
                                                 double* __restrict__ out) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / count;
}

}  // namespace quality

extern "C" foe_status foe_ssim(const float* d_u, const float* d_ref, int32_t H, int32_t W, double peak, void* hip_stream,
                               double* ssim_out) {
  using namespace quality;
  if (!d_u || !d_ref || !ssim_out) {
    foe_internal_set_error("NULL argument");
    return FOE_EINVAL;
  }
  if (H < WIN || W < WIN || !(peak > 0.0) || !std::isfinite(peak)) {
    foe_internal_set_error("SSIM needs images of at least 11 x 11 and a positive peak");
    return FOE_EINVAL;
  }
  hipStream_t stream = (hipStream_t)hip_stream;
  Taps g;
  double sum = 0.0;
  double wd[WIN];
  for (int t = 0; t < WIN; ++t) {
    const double d = t - (WIN - 1) / 2.0;
    wd[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += wd[t];
  }
  for (int t = 0; t < WIN; ++t) g.w[t] = (float)(wd[t] / sum);
  const int Wo = W - WIN + 1, Ho = H - WIN + 1;
  dim3 grid((Wo + TX - 1) / TX, (Ho + TY - 1) / TY);
  const int nb = grid.x * grid.y;
  double* buf = nullptr;
  hipError_t e = hipMalloc(&buf, sizeof(double) * (nb + 1));
  if (e != hipSuccess) {
    foe_internal_set_error(std::string("foe_ssim: ") + hipGetErrorString(e));
    return FOE_ENOMEM;
  }
  const float c1 = (float)((0.01 * peak) * (0.01 * peak)), c2 = (float)((0.03 * peak) * (0.03 * peak));
  ssim_blocks<<<grid, NT, 0, stream>>>(d_u, d_ref, H, W, g, c1, c2, buf + 1);
  ssim_total<<<1, NT, 0, stream>>>(buf + 1, nb, (double)Ho * Wo, buf);
  e = hipGetLastError();
  double host = 0.0;
  if (e == hipSuccess) e = hipMemcpyAsync(&host, buf, sizeof(double), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFree(buf);
  if (e != hipSuccess) {
    foe_internal_set_error(std::string("foe_ssim: ") + hipGetErrorString(e));
    return FOE_EDEVICE;
  }
  *ssim_out = host;
  return FOE_OK;
}
