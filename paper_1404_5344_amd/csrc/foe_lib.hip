// Host runtime and C ABI of the FoE + iPiano library (declared in include/foe.h).
//
// A solver owns one image or a batch of images of uneven sizes, stored as packed planes
// (the images concatenated in index order).  Per solver: the x ring (x^n, x^{n-1},
// candidate), the gradient ring (grad F(x^n), candidate grad F(x+)), a copy of f, the
// flattened list of output tiles over all images, per-tile partial sums, one device iPiano
// state per image and the stats rings.  The iteration loop is a sequence of "slots": one
// fused trial launch over every tile of every image, then one decide launch with one block
// per image.  Decisions live on the device, so the host only synchronises between rounds
// of slots (one round when no trial is rejected); an image whose iterations are done turns
// its tiles into no-ops.  Rounds are replayed from pre-instantiated HIP graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/foe.h"
#include "common.hpp"
#include "kernels_trial.hpp"
#include "kernels_misc.hpp"

using namespace foe;

namespace {

thread_local std::string g_last_error;

foe_status fail(foe_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_OR(expr)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail(FOE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

// Tile configurations of the fused kernel (chosen per solver, by the autotuner if asked).
// V_NT threads per workgroup; the FP32 and split-FP16 matrix-core engines run V_NT_MFMA (16 waves: four per
// SIMD hide the LDS and matrix-pipe latencies better, and their registers fit in the 128 VGPRs that allows).
constexpr int V_NC = 16, V_NT = 512, V_NT_MFMA = 1024, V_BC = 2;
// adjoint register blocks: 4 x 4 outputs on 32 x 32 tiles of the matrix-core kernels, 4 x 2 on 32 x 16 tiles,
// 2 x 2 on 32 x 8 and 64 x 8 tiles (a filter group is a whole number of waves: (TH / BR) (TW / BC) = 64 or 128
// threads)
constexpr int br_for(int th) { return th == 8 ? 2 : 4; }
constexpr int bc_mfma(int th) { return th == 32 ? 4 : V_BC; }
struct TileCfg {
  int tw, th;
};
// 32 x 8 tiles spread small images over more CUs (a 256 x 256 image is 64 tiles of 32 x 32 but 256 of 32 x 8);
// 64 x 8 tiles, half as many, carry less halo per output (76 x 20 / (64 x 8) = 2.97 against 44 x 20 / (32 x 8)
// = 3.44 for 32 x 8).  The BF16 engine's z strips take 32-column tiles of 16-row blocks, so it runs the first
// two only
constexpr TileCfg TILE_CFGS[4] = {{32, 32}, {32, 16}, {32, 8}, {64, 8}};
constexpr int N_TILE_CFGS = 4;
constexpr bool cfg_ok(int cfg, int engine) {
  return !((TILE_CFGS[cfg].th % 16 != 0 || TILE_CFGS[cfg].tw != 32) && engine == 2 /* FWD_MFMA_BF16 */);
}
constexpr int GRAPH_BIG = 16;
static_assert(GRAPH_BIG % 2 == 0, "a big graph must return the state to parity 0");

// The paper's lambda1, lambda2 for L = 1, 3, 8 looks (Sec. III-B); other L are interpolated
// linearly in L and L > 8 takes the L = 8 values.
void paper_lambdas(int looks, double* l1, double* l2) {
  const double T[3][3] = {{1, 160.0, 0.004}, {3, 310.0, 0.008}, {8, 550.0, 0.02}};
  if (looks <= 1) { *l1 = T[0][1]; *l2 = T[0][2]; return; }
  if (looks >= 8) { *l1 = T[2][1]; *l2 = T[2][2]; return; }
  int k = looks < 3 ? 0 : 1;
  double t = (looks - T[k][0]) / (T[k + 1][0] - T[k][0]);
  *l1 = T[k][1] + t * (T[k + 1][1] - T[k][1]);
  *l2 = T[k][2] + t * (T[k + 1][2] - T[k][2]);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Largest |tap| the split-FP16 engine takes: the heads stay below 2^14 and the 4096-scaled tails
// below 2^15, inside the FP16 range.
constexpr float SPLIT_MAX_TAP = 16384.0f;
// The split carries a tap to an absolute resolution of 2^-36 (a head below 2^-14 is an FP16 subnormal):
// relative to a filter whose largest |tap| is at least 2^-10 that is below 2^-26.  AUTO takes the FP32
// engine for a bank with a smaller nonzero filter.
constexpr float SPLIT_MIN_FILTER_MAX = 1.0f / 1024.0f;

// The split-FP16 operands of the forward taps kf ([chunk][t][j], t = 7 a + b): per chunk and lane
// (m = lane % 16, k = lane / 16), for steps s = 0, 1, the heads then the 4096-scaled tails of tap
// row 4s + k, columns 0..7, of filter m (zero outside the 7 x 7 taps), two FP16 per word, the lower
// column in the low half.  out: (MAX_NF / V_NC) * F16_OPS words.
void split_taps(const float* kf, unsigned* out) {
  const int nchunks = MAX_NF / V_NC;
  for (int c = 0; c < nchunks; ++c)
    for (int lane = 0; lane < 64; ++lane) {
      const int m = lane % 16, k = lane / 16;
      for (int s = 0; s < 2; ++s)
        for (int part = 0; part < 2; ++part)
          for (int i = 0; i < 8; i += 2) {
            unsigned short hv[2];
            for (int q = 0; q < 2; ++q) {
              const int ta = 4 * s + k, tb = i + q;
              const float v = ta < KS && tb < KS ? kf[((size_t)c * KK + ta * KS + tb) * V_NC + m] : 0.0f;
              const _Float16 hi = (_Float16)v;
              const _Float16 h = part == 0 ? hi : (_Float16)((v - (float)hi) * 4096.0f);
              hv[q] = __builtin_bit_cast(unsigned short, h);
            }
            out[(size_t)c * F16_OPS + lane * 16 + s * 8 + part * 4 + i / 2] = (unsigned)hv[0] | ((unsigned)hv[1] << 16);
          }
    }
}

// Host copies of every tap table the kernels read, built from the caller's bank (no heap use).
struct TapTables {
  float kf[MAX_NF * KK];                    // forward taps, flipped and chunk-transposed
  float ka[MAX_NF * KK];                    // adjoint taps 2 theta_i k_i
  float theta[MAX_NF];
  unsigned kf16[(MAX_NF / V_NC) * F16_OPS];  // split-FP16 forward operands
  unsigned kb16[MAX_NF * KB16_W];            // BF16 adjoint operands of the BF16 engine's matrix-core adjoint
};

// The BF16 adjoint operands of filter i (ZStrips, KB16_W): T[22 a + b] = ka_i[a][b] (b < 7), zero elsewhere,
// rounded to BF16; copy c holds T[x + c - 16] at half x, two halves per word, the lower index in the low half.
void adjoint_operands_bf16(const float* ka_i, unsigned* out) {
  constexpr int TW_ = 22, NH = 2 * KB16_COPY;
  for (int copy = 0; copy < 2; ++copy)
    for (int x = 0; x < NH; x += 2) {
      unsigned short hv[2];
      for (int q = 0; q < 2; ++q) {
        const int k = x + q + copy - 16;
        const float v = k >= 0 && k < KS * TW_ && k % TW_ < KS ? ka_i[(k / TW_) * KS + k % TW_] : 0.0f;
        hv[q] = __builtin_bit_cast(unsigned short, (__bf16)v);
      }
      out[copy * KB16_COPY + x / 2] = (unsigned)hv[0] | ((unsigned)hv[1] << 16);
    }
}

void build_tap_tables(int nf, const float* filters_host, const float* weights_host, TapTables* t) {
  std::memset(t, 0, sizeof(TapTables));
  for (int i = 0; i < nf; ++i) {
    t->theta[i] = weights_host[i];
    for (int a = 0; a < KS; ++a)
      for (int b = 0; b < KS; ++b) {
        const float k = filters_host[(size_t)i * KK + a * KS + b];
        t->ka[i * KK + a * KS + b] = (float)(2.0 * (double)t->theta[i] * (double)k);   // z planes hold y/(1+y^2)
        const int c = i / V_NC, j = i % V_NC, tt = (KS - 1 - a) * KS + (KS - 1 - b);
        t->kf[((size_t)c * KK + tt) * V_NC + j] = k;
      }
  }
  split_taps(t->kf, t->kf16);
  for (int i = 0; i < nf; ++i) adjoint_operands_bf16(t->ka + i * KK, t->kb16 + (size_t)i * KB16_W);
}

}  // namespace

// Lets the other translation units of the library report through foe_last_error().
void foe_internal_set_error(const std::string& msg) { g_last_error = msg; }

struct foe_solver {
  foe_params p{};
  Problem pb{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int n_img = 0;
  size_t n = 0;  // total pixels
  std::vector<ImageDesc> images;
  std::vector<TileDesc> tiles;
  int tile_cfg = 0;
  int nblocks = 0;
  ImageDesc* d_images = nullptr;
  TileDesc* d_tiles = nullptr;
  float* xr[3] = {nullptr, nullptr, nullptr};
  float* gr[2] = {nullptr, nullptr};
  float* fbuf = nullptr;
  float* scratch = nullptr;  // probe workspace (one packed plane)
  float* zbuf = nullptr;     // unfused path: num_filters packed planes of z
  float* kf = nullptr;
  float* ka = nullptr;
  unsigned* kf16 = nullptr;  // split-FP16 forward operands (FP16 pairs), F16_OPS words per chunk
  unsigned* kb16 = nullptr;  // BF16 adjoint operands, KB16_W words per filter
  float* theta = nullptr;
  double* partials = nullptr;   // per-block partials; partials2 / st2: the other parity of the graph launches
  double* partials2 = nullptr;
  int max_tiles = 0;
  double* stats = nullptr;  // [n_img][max_iters][8]
  int stats_rows = 1;
  DevState* st = nullptr;       // [n_img]
  DevState* st2 = nullptr;      // [n_img]
  DevState* st_host = nullptr;  // pinned mirror [n_img]
  // GRAPH_BIG trial launches from parity 0 (back to parity 0), one launch from parity 0, one from parity 1
  hipGraphExec_t graph_big = nullptr, graph_one = nullptr, graph_one1 = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int last_launches = 0;
};

namespace {

void build_tiles(foe_solver* s, int cfg) {
  const TileCfg tc = TILE_CFGS[cfg];
  s->tiles.clear();
  for (int i = 0; i < s->n_img; ++i) {
    ImageDesc& im = s->images[i];
    im.tile0 = (int)s->tiles.size();
    const int ntx = (im.W + tc.tw - 1) / tc.tw, n = ntx * ((im.H + tc.th - 1) / tc.th);
    for (int b = 0; b < n; ++b) {
      const int t = xcd_tile_order(b, n);
      s->tiles.push_back(TileDesc{i, (t % ntx) * tc.tw, (t / ntx) * tc.th, 0});
    }
    im.ntiles = n;
  }
  s->tile_cfg = cfg;
  s->nblocks = (int)s->tiles.size();
}

foe_status upload_tiles(foe_solver* s) {
  HIP_OR(hipMemcpy(s->d_images, s->images.data(), sizeof(ImageDesc) * s->n_img, hipMemcpyHostToDevice));
  HIP_OR(hipMemcpy(s->d_tiles, s->tiles.data(), sizeof(TileDesc) * s->nblocks, hipMemcpyHostToDevice));
  return FOE_OK;
}

FusedArgs fused_args(foe_solver* s, int mode, const float* f, const float* x_in, float* g_out) {
  FusedArgs a;
  a.pb = s->pb;
  a.tiles = s->d_tiles;
  a.images = s->d_images;
  a.f = f;
  a.xr0 = s->xr[0]; a.xr1 = s->xr[1]; a.xr2 = s->xr[2];
  a.gr0 = s->gr[0]; a.gr1 = s->gr[1];
  a.x_in = x_in;
  a.g_out = g_out;
  a.st = s->st;
  a.partials = s->partials;
  a.decide_prev = 0;
  a.st_out = nullptr;
  a.part_in = nullptr;
  a.stats = s->stats;
  a.stats_rows = s->stats_rows;
  a.kf = s->kf;
  a.ka = s->ka;
  a.kf16 = s->kf16;
  a.kb16 = s->kb16;
  a.theta = s->theta;
  a.zbuf = s->zbuf;
  a.zstride = (long long)s->n;
  a.mode = mode;
  return a;
}

template <int TW, int TH, int UNF>
void launch_engine(foe_solver* s, const FusedArgs& a, hipStream_t stream) {
  constexpr int BR = br_for(TH);
  if (s->pb.engine == FWD_MFMA_BF16) {
    if constexpr (TH % 16 == 0 && TW == 32)   // cfg_ok keeps the BF16 engine off other tile shapes
      foe_trial_kernel<TW, TH, V_NC, V_NT_MFMA, BR, bc_mfma(TH), FWD_MFMA_BF16, UNF><<<s->nblocks, V_NT_MFMA, 0, stream>>>(a);
  } else if (s->pb.engine == FWD_MFMA_F32) {
    foe_trial_kernel<TW, TH, V_NC, V_NT_MFMA, BR, bc_mfma(TH), FWD_MFMA_F32, UNF><<<s->nblocks, V_NT_MFMA, 0, stream>>>(a);
  } else if (s->pb.engine == FWD_MFMA_F16X) {
    foe_trial_kernel<TW, TH, V_NC, V_NT_MFMA, BR, bc_mfma(TH), FWD_MFMA_F16X, UNF><<<s->nblocks, V_NT_MFMA, 0, stream>>>(a);
  } else {
    foe_trial_kernel<TW, TH, V_NC, V_NT, BR, V_BC, FWD_VALU, UNF><<<s->nblocks, V_NT, 0, stream>>>(a);
  }
}

// One trial (or evaluation): the fused kernel, or its two halves exchanging z through HBM.
template <int TW, int TH>
void launch_cfg(foe_solver* s, const FusedArgs& a, hipStream_t stream) {
  if (s->zbuf) {
    launch_engine<TW, TH, FWD_HALF>(s, a, stream);
    // the adjoint half runs no forward bank; it takes the adjoint form and thread count of the engine's fused
    // kernel, so that both paths compute the adjoint with the same arithmetic in the same order
    constexpr int BR = br_for(TH);
    if (s->pb.engine == FWD_MFMA_BF16) {
      if constexpr (TH % 16 == 0 && TW == 32)
        foe_trial_kernel<TW, TH, V_NC, V_NT_MFMA, BR, bc_mfma(TH), FWD_MFMA_BF16, ADJ_HALF><<<s->nblocks, V_NT_MFMA, 0, stream>>>(a);
    } else if (s->pb.engine == FWD_MFMA_F32 || s->pb.engine == FWD_MFMA_F16X) {
      foe_trial_kernel<TW, TH, V_NC, V_NT_MFMA, BR, bc_mfma(TH), FWD_VALU, ADJ_HALF><<<s->nblocks, V_NT_MFMA, 0, stream>>>(a);
    } else {
      foe_trial_kernel<TW, TH, V_NC, V_NT, BR, V_BC, FWD_VALU, ADJ_HALF><<<s->nblocks, V_NT, 0, stream>>>(a);
    }
  } else {
    launch_engine<TW, TH, FUSED>(s, a, stream);
  }
}

void launch_fused(foe_solver* s, const FusedArgs& a, hipStream_t stream) {
  if (s->tile_cfg == 3)
    launch_cfg<64, 8>(s, a, stream);
  else if (s->tile_cfg == 2)
    launch_cfg<32, 8>(s, a, stream);
  else if (s->tile_cfg == 1)
    launch_cfg<32, 16>(s, a, stream);
  else
    launch_cfg<32, 32>(s, a, stream);
}

void launch_decide(foe_solver* s, int mode, hipStream_t stream, int parity = 0) {
  decide_kernel<<<s->n_img, 256, 0, stream>>>(parity ? s->st2 : s->st, parity ? s->partials2 : s->partials, s->d_images,
                                              s->pb, s->stats, s->stats_rows, mode);
}

dim3 grid_img(const foe_solver* s) {
  size_t mx = 0;
  for (const ImageDesc& im : s->images) mx = std::max(mx, (size_t)im.H * im.W);
  size_t b = (mx + 255) / 256;
  return dim3((unsigned)std::min<size_t>(std::max<size_t>(b, 1), 1024), (unsigned)s->n_img, 1);
}

int grid_1d(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

// Validates the parameters shared by every image and fills the shared Problem.
foe_status validate(const foe_params* p, const float* filters, const float* weights, Problem* pb) {
  if (!p) return fail(FOE_EINVAL, "params is NULL");
  if (!filters || !weights) return fail(FOE_EINVAL, "filters/weights is NULL");
  if (p->num_filters < 1 || p->num_filters > FOE_MAX_FILTERS) return fail(FOE_EINVAL, "num_filters out of range");
  if (p->ksize != FOE_KSIZE) return fail(FOE_EINVAL, "ksize must be 7");
  if (p->model < 0 || p->model > 2) return fail(FOE_EINVAL, "bad model");
  if (p->boundary < 0 || p->boundary > 2) return fail(FOE_EINVAL, "bad boundary");
  if (p->precision != FOE_PREC_FP32 && p->precision != FOE_PREC_BF16) return fail(FOE_EINVAL, "bad precision");
  if (p->engine < FOE_ENGINE_AUTO || p->engine > FOE_ENGINE_MFMA_SPLIT) return fail(FOE_EINVAL, "bad engine");
  if (p->fusion != FOE_FUSED && p->fusion != FOE_UNFUSED) return fail(FOE_EINVAL, "bad fusion");
  if (p->prox_method != FOE_PROX_NEWTON && p->prox_method != FOE_PROX_LAMBERTW) return fail(FOE_EINVAL, "bad prox_method");
  if (p->prox_method == FOE_PROX_LAMBERTW && p->model != FOE_MODEL_LOG)
    return fail(FOE_EINVAL, "the Lambert-W prox exists for the LOG model only");
  if (p->precision == FOE_PREC_BF16 && p->engine != FOE_ENGINE_AUTO)
    return fail(FOE_EINVAL, "BF16 precision runs its own engine (engine must be AUTO)");
  if (p->step_mode != FOE_STEP_BACKTRACK && p->step_mode != FOE_STEP_FIXED) return fail(FOE_EINVAL, "bad step_mode");
  if (p->max_iters < 0) return fail(FOE_EINVAL, "max_iters must be >= 0");
  if (p->max_backtracks < 0) return fail(FOE_EINVAL, "max_backtracks must be >= 0");
  if (p->newton_iters < 1 || p->newton_iters > 100) return fail(FOE_EINVAL, "newton_iters must be in [1, 100]");
  if (!(p->beta >= 0.0 && p->beta < 1.0)) return fail(FOE_EINVAL, "beta must be in [0, 1)");
  if (p->step_mode == FOE_STEP_FIXED && !finite_pos(p->alpha_fixed)) return fail(FOE_EINVAL, "alpha_fixed must be > 0");
  if (p->step_mode == FOE_STEP_BACKTRACK) {
    if (!finite_pos(p->L0)) return fail(FOE_EINVAL, "L0 must be > 0");
    if (!(std::isfinite(p->eta_up) && p->eta_up > 1.0)) return fail(FOE_EINVAL, "eta_up must be > 1");
    if (!(p->eta_down > 0.0 && p->eta_down <= 1.0)) return fail(FOE_EINVAL, "eta_down must be in (0, 1]");
  }
  bool split_ok = true, split_fine = true;
  for (int i = 0; i < p->num_filters * FOE_KSIZE * FOE_KSIZE; ++i) {
    if (!std::isfinite(filters[i])) return fail(FOE_EINVAL, "non-finite filter tap");
    if (!(std::fabs(filters[i]) < SPLIT_MAX_TAP)) split_ok = false;
  }
  for (int j = 0; j < p->num_filters; ++j) {
    float mx = 0.0f;
    for (int t = 0; t < FOE_KSIZE * FOE_KSIZE; ++t) mx = std::max(mx, std::fabs(filters[j * FOE_KSIZE * FOE_KSIZE + t]));
    if (mx > 0.0f && mx < SPLIT_MIN_FILTER_MAX) split_fine = false;
  }
  if ((p->engine == FOE_ENGINE_MFMA_SPLIT || p->precision == FOE_PREC_BF16) && !split_ok)
    return fail(FOE_EINVAL, "the split-FP16 engine (also the forward of BF16 precision) takes taps with |k| < 16384");
  for (int i = 0; i < p->num_filters; ++i)
    if (!(std::isfinite(weights[i]) && weights[i] >= 0.0f)) return fail(FOE_EINVAL, "weights must be finite, >= 0");
  pb->nf = p->num_filters;
  pb->model = p->model;
  pb->bc = p->boundary;
  pb->step_mode = p->step_mode;
  pb->max_backtracks = p->max_backtracks;
  pb->newton_iters = p->newton_iters;
  pb->prox_method = p->prox_method;
  pb->beta = (float)p->beta;
  pb->beta_d = p->beta;
  pb->eta_up = p->eta_up;
  pb->eta_down = p->eta_down;
  pb->alpha_fixed = p->alpha_fixed;
  if (p->precision == FOE_PREC_BF16)
    pb->engine = FWD_MFMA_BF16;
  else if (p->engine == FOE_ENGINE_VALU)
    pb->engine = FWD_VALU;
  else if (p->engine == FOE_ENGINE_MFMA)
    pb->engine = FWD_MFMA_F32;
  else if (p->engine == FOE_ENGINE_MFMA_SPLIT)
    pb->engine = FWD_MFMA_F16X;
  else   // AUTO: the split engine unless a tap is out of its range or a filter is below its resolution
    pb->engine = split_ok && split_fine ? FWD_MFMA_F16X : FWD_MFMA_F32;
  return FOE_OK;
}

// Per-image size and data-term weights (lambda < 0 => the paper's value for `looks`).
foe_status image_desc(const foe_params* p, int H, int W, double l1, double l2, int looks, ImageDesc* im) {
  if (H < 4 || W < 4) return fail(FOE_EINVAL, "height and width must be >= 4");
  if ((int64_t)H * W > ((int64_t)1 << 31)) return fail(FOE_EINVAL, "image too large");
  if (looks < 1) return fail(FOE_EINVAL, "looks must be >= 1");
  if (p->model == FOE_MODEL_IDIV) {
    if (!(std::isfinite(l1) && l1 >= 0.0)) return fail(FOE_EINVAL, "IDIV needs lambda1 >= 0");
  } else {
    double d1, d2;
    paper_lambdas(looks, &d1, &d2);
    if (l1 < 0.0) l1 = d1;
    if (l2 < 0.0) l2 = d2;
    if (!std::isfinite(l1) || !std::isfinite(l2)) return fail(FOE_EINVAL, "lambda must be finite");
  }
  if (p->model != FOE_MODEL_COMBINED) l2 = 0.0;
  im->H = H;
  im->W = W;
  im->lam1 = (float)l1;
  im->lam2 = (float)l2;
  return FOE_OK;
}

void destroy_all(foe_solver* s) {
  if (!s) return;
  if (s->graph_big) (void)hipGraphExecDestroy(s->graph_big);
  if (s->graph_one) (void)hipGraphExecDestroy(s->graph_one);
  if (s->graph_one1) (void)hipGraphExecDestroy(s->graph_one1);
  for (float* p : s->xr) if (p) (void)hipFree(p);
  for (float* p : s->gr) if (p) (void)hipFree(p);
  void* bufs[] = {s->fbuf, s->scratch, s->zbuf, s->kf, s->ka, s->kf16, s->kb16, s->theta, s->partials, s->partials2, s->stats, s->st, s->st2,
                  s->d_images, s->d_tiles};
  for (void* b : bufs) if (b) (void)hipFree(b);
  if (s->st_host) (void)hipHostFree(s->st_host);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

void drop_graphs(foe_solver* s) {
  if (s->graph_big) (void)hipGraphExecDestroy(s->graph_big);
  if (s->graph_one) (void)hipGraphExecDestroy(s->graph_one);
  if (s->graph_one1) (void)hipGraphExecDestroy(s->graph_one1);
  s->graph_big = s->graph_one = s->graph_one1 = nullptr;
}

// A graph of `slots` trial launches starting at `parity`: launch n reads the state and the partials of
// parity (parity + n) % 2, decides the previous trial in every workgroup, runs its own trial and writes
// the state and the partials of the other parity.  No separate decision launch between trials.
foe_status build_graph(foe_solver* s, int slots, int parity, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_OR(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < slots; ++k) {
    const int q = (parity + k) & 1;
    FusedArgs a = fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr);
    a.decide_prev = 1;
    a.st = q ? s->st2 : s->st;
    a.st_out = q ? s->st : s->st2;
    a.part_in = q ? s->partials2 : s->partials;
    a.partials = q ? s->partials : s->partials2;
    launch_fused(s, a, s->cap_stream);
  }
  HIP_OR(hipStreamEndCapture(s->cap_stream, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(FOE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return FOE_OK;
}

// Host-side initial device state of every image for a launch sequence of `iters` iterations
// from ring slots 0 (x^n) and 1 (x^{n-1}).
void reset_states(foe_solver* s, const double* L_in, int iters) {
  for (int i = 0; i < s->n_img; ++i) {
    DevState& h = s->st_host[i];
    std::memset(&h, 0, sizeof(DevState));
    h.icur = 0; h.iprev = 1; h.icand = 2;
    h.gcur = 0; h.gcand = 1;
    h.target = iters;
    if (s->pb.step_mode == FIXED) {
      h.L = L_in[i];
      h.alpha = s->pb.alpha_fixed;
    } else {
      h.L = s->pb.eta_down * L_in[i];
      h.alpha = 1.9 * (1.0 - s->pb.beta_d) / h.L;
    }
    h.L_acc = L_in[i];
  }
}

foe_status push_states(foe_solver* s) {
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState) * s->n_img, hipMemcpyHostToDevice, s->stream));
  return FOE_OK;
}

foe_status pull_states(foe_solver* s) {
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState) * s->n_img, hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  return FOE_OK;
}

foe_status status_of(int st) {
  switch (st) {
    case ST_OK: return FOE_OK;
    case ST_ELINESEARCH: return fail(FOE_ELINESEARCH, "backtracking exceeded max_backtracks");
    case ST_ENONFINITE: return fail(FOE_ENONFINITE, "non-finite energy or reduction");
    case ST_EINPUT: return fail(FOE_EINPUT, "f or the initial image has a non-finite or non-positive pixel");
    default: return fail(FOE_EDEVICE, "unknown device status");
  }
}

// Runs the iteration loop of every image from ring slots 0 / 1; fbuf holds f.  Summaries and
// stats are per image.  Returns the first image's failure status, if any.
// The iteration loop from the ring state (x^0 in slot 0, x^{-1} in slot 1).  pre (nullable) is launched on
// the stream after the state upload and before the evaluation at x^0: the input check, which sets
// input_bad; then the first state download, which the loop needs anyway, also reports the check (the
// decision at x^0 marks such an image done), and the call returns EINPUT without iterating.  Each round
// launches the trials still missing plus a few more (at least GRAPH_BIG), so that rejected trials seldom
// cost a second round (a trial launch after an image is done leaves it unchanged).
template <class Pre>
foe_status run_loop(foe_solver* s, const double* L_in, int iters, foe_summary* sums, double* stats_host, Pre pre) {
  reset_states(s, L_in, iters);
  foe_status e = push_states(s);
  if (e != FOE_OK) return e;
  pre();
  // F, G and grad F at x^0
  launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
  launch_decide(s, DECIDE_INIT, s->stream);
  HIP_OR(hipGetLastError());
  if (!s->graph_big) {
    e = build_graph(s, GRAPH_BIG, 0, &s->graph_big);
    if (e != FOE_OK) return e;
    e = build_graph(s, 1, 0, &s->graph_one);
    if (e != FOE_OK) return e;
    e = build_graph(s, 1, 1, &s->graph_one1);
    if (e != FOE_OK) return e;
  }
  HIP_OR(hipEventRecord(s->ev0, s->stream));
  e = pull_states(s);
  if (e != FOE_OK) return e;
  bool bad = false;
  for (int i = 0; i < s->n_img; ++i) bad = bad || s->st_host[i].input_bad;
  if (bad) {
    if (sums) std::memset(sums, 0, sizeof(foe_summary) * s->n_img);
    return fail(FOE_EINPUT, "f or the initial image has a non-finite or non-positive pixel");
  }
  std::vector<double> G0(s->n_img);
  for (int i = 0; i < s->n_img; ++i) G0[i] = s->st_host[i].sums[1];
  for (;;) {
    int remaining = 0;
    for (int i = 0; i < s->n_img; ++i) {
      const DevState& h = s->st_host[i];
      if (!h.done) remaining = std::max(remaining, h.target - h.iter);
    }
    if (remaining <= 0) break;
    // at least one big graph: a short solve from a far L0 (ten or more rejections in its first iteration)
    // still ends in one round
    const int n_launch = std::max(GRAPH_BIG, remaining + remaining / 16 + 1);
    // the state and partials start at parity 0; GRAPH_BIG is even, so each big graph ends at parity 0
    int q = 0;
    for (int k = 0; k < n_launch / GRAPH_BIG; ++k) HIP_OR(hipGraphLaunch(s->graph_big, s->stream));
    for (int k = 0; k < n_launch % GRAPH_BIG; ++k) {
      HIP_OR(hipGraphLaunch(q ? s->graph_one1 : s->graph_one, s->stream));
      q ^= 1;
    }
    // the decision on the last trial, then the state back to parity 0
    launch_decide(s, DECIDE_STEP, s->stream, q);
    if (q) HIP_OR(hipMemcpyAsync(s->st, s->st2, sizeof(DevState) * s->n_img, hipMemcpyDeviceToDevice, s->stream));
    e = pull_states(s);
    if (e != FOE_OK) return e;
  }
  HIP_OR(hipEventRecord(s->ev1, s->stream));
  HIP_OR(hipEventSynchronize(s->ev1));
  float ms = 0.f;
  HIP_OR(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  s->last_ms = ms;
  // launches that ran a trial: one per trial of the image with the most trials (the others are no-ops)
  int launches = 0;
  for (int i = 0; i < s->n_img; ++i) launches = std::max(launches, s->st_host[i].total_trials);
  s->last_launches = launches;
  std::vector<double> rows;
  if (stats_host || sums) {
    rows.resize((size_t)s->n_img * s->stats_rows * STAT_COLS);
    HIP_OR(hipMemcpy(rows.data(), s->stats, sizeof(double) * rows.size(), hipMemcpyDeviceToHost));
  }
  foe_status first = FOE_OK;
  for (int i = 0; i < s->n_img; ++i) {
    const DevState& h = s->st_host[i];
    const double* ri = rows.empty() ? nullptr : rows.data() + (size_t)i * s->stats_rows * STAT_COLS;
    if (stats_host && h.iter > 0)
      std::memcpy(stats_host + (size_t)i * s->stats_rows * STAT_COLS, ri, sizeof(double) * STAT_COLS * h.iter);
    if (sums) {
      foe_summary& sm = sums[i];
      sm.iters_done = h.iter;
      sm.total_trials = h.total_trials;
      sm.F = h.Fcur;
      sm.G = h.iter > 0 ? ri[(size_t)(h.iter - 1) * STAT_COLS + 1] : G0[i];
      sm.alpha = h.iter > 0 ? ri[(size_t)(h.iter - 1) * STAT_COLS + 3] : h.alpha;
      sm.H = sm.F + sm.G;
      sm.L = h.L_acc;
    }
    if (h.status != ST_OK && first == FOE_OK) first = status_of(h.status);
  }
  return first;
}

foe_status create_common(const foe_params* p, int n_img, const int32_t* H, const int32_t* W, const double* l1,
                         const double* l2, const int32_t* looks, const float* filters_host,
                         const float* weights_host, void* hip_stream, foe_solver** out) {
  if (!out) return fail(FOE_EINVAL, "out is NULL");
  if (n_img < 1) return fail(FOE_EINVAL, "need at least one image");
  Problem pb;
  foe_status v = validate(p, filters_host, weights_host, &pb);
  if (v != FOE_OK) return v;
  std::vector<ImageDesc> images(n_img);
  long long off = 0;
  for (int i = 0; i < n_img; ++i) {
    v = image_desc(p, H[i], W[i], l1[i], l2[i], looks[i], &images[i]);
    if (v != FOE_OK) return v;
    images[i].off = off;
    off += (long long)H[i] * W[i];
  }
  foe_solver* s = new (std::nothrow) foe_solver();
  if (!s) return fail(FOE_ENOMEM, "host allocation failed");
  s->p = *p;
  s->pb = pb;
  s->stream = (hipStream_t)hip_stream;
  s->n_img = n_img;
  s->n = (size_t)off;
  s->images = images;
  // the tile list of the configuration with the most tiles bounds the partials buffer
  for (int c = 0; c < N_TILE_CFGS; ++c) {
    build_tiles(s, c);
    s->max_tiles = std::max(s->max_tiles, s->nblocks);
  }
  build_tiles(s, 0);
  s->stats_rows = p->max_iters > 0 ? p->max_iters : 1;
  const size_t plane = sizeof(float) * s->n;
  std::string alloc_err;
  auto alloc = [&](void** ptr, size_t bytes) -> bool {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) alloc_err = std::to_string(bytes) + " bytes: " + hipGetErrorString(e);
    return e == hipSuccess;
  };
  bool ok = true;
  for (auto& x : s->xr) ok = ok && alloc((void**)&x, plane);
  for (auto& g : s->gr) ok = ok && alloc((void**)&g, plane);
  ok = ok && alloc((void**)&s->fbuf, plane) && alloc((void**)&s->scratch, plane);
  if (p->fusion == FOE_UNFUSED) ok = ok && alloc((void**)&s->zbuf, plane * p->num_filters);
  ok = ok && alloc((void**)&s->kf, sizeof(float) * MAX_NF * KK) && alloc((void**)&s->ka, sizeof(float) * MAX_NF * KK);
  ok = ok && alloc((void**)&s->kf16, sizeof(unsigned) * (MAX_NF / V_NC) * F16_OPS);
  ok = ok && alloc((void**)&s->kb16, sizeof(unsigned) * MAX_NF * KB16_W);
  ok = ok && alloc((void**)&s->theta, sizeof(float) * MAX_NF);
  ok = ok && alloc((void**)&s->partials, sizeof(double) * PART_COLS * (size_t)s->max_tiles);
  ok = ok && alloc((void**)&s->partials2, sizeof(double) * PART_COLS * (size_t)s->max_tiles);
  ok = ok && alloc((void**)&s->stats, sizeof(double) * STAT_COLS * (size_t)s->stats_rows * n_img);
  ok = ok && alloc((void**)&s->st, sizeof(DevState) * n_img) && alloc((void**)&s->st2, sizeof(DevState) * n_img);
  ok = ok && alloc((void**)&s->d_images, sizeof(ImageDesc) * n_img);
  ok = ok && alloc((void**)&s->d_tiles, sizeof(TileDesc) * (size_t)s->max_tiles);
  ok = ok && hipHostMalloc((void**)&s->st_host, sizeof(DevState) * n_img, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    destroy_all(s);
    return fail(FOE_ENOMEM, "device allocation failed (" + alloc_err + ")");
  }
  std::unique_ptr<TapTables> tabs(new (std::nothrow) TapTables);
  if (!tabs) {
    destroy_all(s);
    return fail(FOE_ENOMEM, "host allocation failed");
  }
  build_tap_tables(p->num_filters, filters_host, weights_host, tabs.get());
  hipError_t e = hipMemcpy(s->kf, tabs->kf, sizeof(tabs->kf), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->kf16, tabs->kf16, sizeof(tabs->kf16), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->ka, tabs->ka, sizeof(tabs->ka), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->kb16, tabs->kb16, sizeof(tabs->kb16), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->theta, tabs->theta, sizeof(tabs->theta), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&s->ev0);
  if (e == hipSuccess) e = hipEventCreate(&s->ev1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    destroy_all(s);
    return fail(FOE_EDEVICE, std::string("foe_create: ") + hipGetErrorString(e));
  }
  v = upload_tiles(s);
  if (v != FOE_OK) {
    destroy_all(s);
    return v;
  }
  *out = s;
  return FOE_OK;
}

foe_status init_from_f(foe_solver* s, const float* d_f, const float* d_u0, bool* bad) {
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  std::vector<double> L(s->n_img, s->p.L0);
  reset_states(s, L.data(), s->p.max_iters);  // ring slot 0 = x^0 even if the input is rejected
  foe_status e = push_states(s);
  if (e != FOE_OK) return e;
  init_state_kernel<<<grid_img(s), 256, 0, s->stream>>>(s->fbuf, d_u0, s->xr[0], s->xr[1], s->d_images,
                                                        s->pb.model, s->st);
  HIP_OR(hipGetLastError());
  e = pull_states(s);
  if (e != FOE_OK) return e;
  *bad = false;
  for (int i = 0; i < s->n_img; ++i) *bad = *bad || s->st_host[i].input_bad;
  return FOE_OK;
}

// Key of the autotuner cache: engine, boundary, filter count, fusion, and the size bucket of the work: the
// number of 32 x 32 tiles of all images, rounded up to a power of two (the tile shapes differ in how well
// they fill the 256 CUs, which that count decides), and whether the batch holds one image or several.
std::string tune_key(const foe_solver* s) {
  long long tiles = 0;
  for (const ImageDesc& im : s->images) tiles += (long long)((im.H + 31) / 32) * ((im.W + 31) / 32);
  int b = 0;
  while ((1ll << b) < tiles) ++b;
  std::ostringstream o;
  o << "e" << s->pb.engine << "_bc" << s->pb.bc << "_nf" << s->pb.nf << "_u" << (s->zbuf ? 1 : 0) << "_t2^" << b
    << (s->n_img > 1 ? "_batch" : "_single");
  return o.str();
}

}  // namespace

extern "C" {

void foe_default_params(foe_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->num_filters = 48;
  p->ksize = FOE_KSIZE;
  p->model = FOE_MODEL_COMBINED;
  p->boundary = FOE_BC_SYMMETRIC;
  p->precision = FOE_PREC_FP32;
  p->step_mode = FOE_STEP_BACKTRACK;
  p->looks = 1;
  p->max_iters = 300;
  p->max_backtracks = 40;
  p->newton_iters = 30;
  p->engine = FOE_ENGINE_AUTO;
  p->fusion = FOE_FUSED;
  p->prox_method = FOE_PROX_NEWTON;
  p->lambda1 = -1.0;
  p->lambda2 = -1.0;
  p->beta = 0.8;
  p->alpha_fixed = 0.0;
  p->L0 = 1.0;
  p->eta_up = 2.0;
  p->eta_down = 1.0;
}

foe_status foe_create(const foe_params* p, const float* filters_host, const float* weights_host, void* hip_stream,
                      foe_solver** out) {
  if (!p) return fail(FOE_EINVAL, "params is NULL");
  const int32_t H = p->height, W = p->width, L = p->looks;
  const double l1 = p->lambda1, l2 = p->lambda2;
  return create_common(p, 1, &H, &W, &l1, &l2, &L, filters_host, weights_host, hip_stream, out);
}

foe_status foe_batch_create(const foe_params* shared, int32_t n, const int32_t* heights, const int32_t* widths,
                            const double* lambda1, const double* lambda2, const int32_t* looks,
                            const float* filters_host, const float* weights_host, void* hip_stream,
                            foe_solver** out) {
  if (!shared || !heights || !widths || !looks) return fail(FOE_EINVAL, "NULL argument");
  if (n < 1 || n > 65535) return fail(FOE_EINVAL, "batch size must be in [1, 65535]");
  std::vector<double> l1(n, -1.0), l2(n, -1.0);
  for (int i = 0; i < n; ++i) {
    if (lambda1) l1[i] = lambda1[i];
    if (lambda2) l2[i] = lambda2[i];
  }
  return create_common(shared, n, heights, widths, l1.data(), l2.data(), looks, filters_host, weights_host,
                       hip_stream, out);
}

foe_status foe_batch_layout(foe_solver* s, int32_t* n_images, int64_t* offsets_host) {
  if (!s) return fail(FOE_EINVAL, "solver is NULL");
  if (n_images) *n_images = s->n_img;
  if (offsets_host) {
    for (int i = 0; i < s->n_img; ++i) offsets_host[i] = s->images[i].off;
    offsets_host[s->n_img] = (int64_t)s->n;
  }
  return FOE_OK;
}

foe_status foe_destroy(foe_solver* s) {
  if (!s) return fail(FOE_EINVAL, "solver is NULL");
  (void)hipStreamSynchronize(s->stream);
  destroy_all(s);
  return FOE_OK;
}

foe_status foe_batch_solve(foe_solver* s, const float* d_f, const float* d_init, float* d_u_out,
                           foe_summary* sums_host, double* stats_host) {
  if (!s || !d_f || !d_u_out) return fail(FOE_EINVAL, "NULL argument");
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  std::vector<double> L(s->n_img, s->p.L0);
  // ring slot 0 = x^0 (from f or d_init) even if the input is rejected
  foe_status st = run_loop(s, L.data(), s->p.max_iters, sums_host, stats_host, [&] {
    init_state_kernel<<<grid_img(s), 256, 0, s->stream>>>(s->fbuf, d_init, s->xr[0], s->xr[1], s->d_images,
                                                          s->pb.model, s->st);
  });
  finalize_kernel<<<grid_img(s), 256, 0, s->stream>>>(s->st, s->xr[0], s->xr[1], s->xr[2], d_u_out, s->d_images,
                                                      s->pb.model);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  return st;
}

foe_status foe_solve(foe_solver* s, const float* d_f, const float* d_init, float* d_u_out, foe_summary* sum_host,
                     double* stats_host) {
  if (s && s->n_img != 1) return fail(FOE_EINVAL, "batch solver: use foe_batch_solve");
  return foe_batch_solve(s, d_f, d_init, d_u_out, sum_host, stats_host);
}

foe_status foe_solve_from(foe_solver* s, const float* d_f, float* d_x_cur, float* d_x_prev, double* L_inout,
                          int32_t iters, foe_summary* sum_host, double* stats_host) {
  if (!s || !d_f || !d_x_cur || !d_x_prev || !L_inout) return fail(FOE_EINVAL, "NULL argument");
  if (iters < 0 || iters > s->p.max_iters) return fail(FOE_EINVAL, "iters must be in [0, max_iters]");
  for (int i = 0; i < s->n_img; ++i)
    if (!finite_pos(L_inout[i])) return fail(FOE_EINVAL, "L must be > 0");
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[0], d_x_cur, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[1], d_x_prev, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  foe_status st = run_loop(s, L_inout, iters, sum_host, stats_host, [&] {
    check_input_kernel<<<grid_img(s), 256, 0, s->stream>>>(s->fbuf, s->d_images, s->st);
  });
  if (st == FOE_EINPUT) return st;   // the state is left as it was
  export_state_kernel<<<grid_img(s), 256, 0, s->stream>>>(s->st, s->xr[0], s->xr[1], s->xr[2], d_x_cur, d_x_prev,
                                                          s->d_images);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  for (int i = 0; i < s->n_img; ++i) L_inout[i] = s->st_host[i].L_acc;
  return st;
}

foe_status foe_eval_gradient(foe_solver* s, const float* d_x, float* d_grad) {
  if (!s || !d_x || !d_grad) return fail(FOE_EINVAL, "NULL argument");
  // G is not reported; f = x keeps the data-term arithmetic finite
  launch_fused(s, fused_args(s, MODE_EVAL, d_x, d_x, d_grad), s->stream);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  return FOE_OK;
}

foe_status foe_eval_energy(foe_solver* s, const float* d_x, const float* d_f, double* F, double* G) {
  if (!s || !d_x || !d_f) return fail(FOE_EINVAL, "NULL argument");
  launch_fused(s, fused_args(s, MODE_EVAL, d_f, d_x, s->scratch), s->stream);
  launch_decide(s, DECIDE_REPORT, s->stream);
  HIP_OR(hipGetLastError());
  foe_status e = pull_states(s);
  if (e != FOE_OK) return e;
  for (int i = 0; i < s->n_img; ++i) {
    if (F) F[i] = s->st_host[i].sums[0];
    if (G) G[i] = s->st_host[i].sums[1];
  }
  return FOE_OK;
}

foe_status foe_eval_prox(foe_solver* s, const float* d_xhat, const float* d_f, double tau, float* d_out) {
  if (!s || !d_xhat || !d_f || !d_out) return fail(FOE_EINVAL, "NULL argument");
  if (s->n_img != 1) return fail(FOE_EINVAL, "prox probe takes a single-image solver");
  if (!finite_pos(tau)) return fail(FOE_EINVAL, "tau must be > 0");
  prox_probe_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(d_xhat, d_f, d_out, s->n, (float)tau, s->pb,
                                                          s->images[0].lam1, s->images[0].lam2);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  return FOE_OK;
}

foe_status foe_step(foe_solver* s, const float* d_f, const float* d_x, const float* d_xprev, double L_forced,
                    float* d_xnext, double* info_host) {
  if (!s || !d_f || !d_x || !d_xprev || !d_xnext) return fail(FOE_EINVAL, "NULL argument");
  if (s->n_img != 1) return fail(FOE_EINVAL, "step probe takes a single-image solver");
  if (s->pb.step_mode == BACKTRACK && !finite_pos(L_forced)) return fail(FOE_EINVAL, "L_forced must be > 0");
  // ring: slot 0 = x, slot 1 = xprev, slot 2 = output; gradient of x into gr[0]
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[0], d_x, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[1], d_xprev, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
  DevState& h = s->st_host[0];
  std::memset(&h, 0, sizeof(DevState));
  h.icur = 0; h.iprev = 1; h.icand = 2; h.gcur = 0; h.gcand = 1; h.target = 1;
  h.L = L_forced;
  h.alpha = s->pb.step_mode == FIXED ? s->pb.alpha_fixed : 1.9 * (1.0 - s->pb.beta_d) / L_forced;
  foe_status e = push_states(s);
  if (e != FOE_OK) return e;
  launch_fused(s, fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr), s->stream);
  launch_decide(s, DECIDE_REPORT, s->stream);
  HIP_OR(hipGetLastError());
  HIP_OR(hipMemcpyAsync(d_xnext, s->xr[2], sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  e = pull_states(s);
  if (e != FOE_OK) return e;
  if (info_host) {
    info_host[0] = h.sums[0];
    info_host[1] = h.sums[1];
    info_host[2] = h.sums[2];
    info_host[3] = h.sums[3];
  }
  return FOE_OK;
}

foe_status foe_last_timing(foe_solver* s, double* ms, int32_t* trial_launches) {
  if (!s) return fail(FOE_EINVAL, "solver is NULL");
  if (ms) *ms = s->last_ms;
  if (trial_launches) *trial_launches = s->last_launches;
  return FOE_OK;
}

foe_status foe_batch_latency(foe_solver* s, double* ms_host) {
  if (!s || !ms_host) return fail(FOE_EINVAL, "NULL argument");
  int dev = 0, khz = 0;
  HIP_OR(hipGetDevice(&dev));
  HIP_OR(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(FOE_EDEVICE, "the device reports no wall-clock rate");
  for (int i = 0; i < s->n_img; ++i) {
    const DevState& h = s->st_host[i];
    ms_host[i] = h.t_done > 0 && h.t_start > 0 ? (double)(h.t_done - h.t_start) / (double)khz : -1.0;
  }
  return FOE_OK;
}

foe_status foe_real_sar_params(foe_params* p) {
  if (!p) return fail(FOE_EINVAL, "NULL argument");
  foe_default_params(p);
  p->looks = 5;
  p->lambda1 = 50.0;
  p->lambda2 = 0.15;
  return FOE_OK;
}

foe_status foe_profile_trial(foe_solver* s, int32_t reps, double* ms_mean) {
  if (!s || reps < 1 || !ms_mean) return fail(FOE_EINVAL, "bad argument");
  if (!s->graph_big) return fail(FOE_EINVAL, "run foe_solve first");
  foe_status st = pull_states(s);
  if (st != FOE_OK) return st;
  std::vector<DevState> saved(s->st_host, s->st_host + s->n_img);
  for (int i = 0; i < s->n_img; ++i) s->st_host[i].done = 0;
  st = push_states(s);
  if (st != FOE_OK) return st;
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) st = fail(FOE_EDEVICE, "hipEventCreate failed");
  const FusedArgs a = fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr);
  double total = 0.0;
  if (st == FOE_OK) {
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(ev[2 * r], s->stream);
      launch_fused(s, a, s->stream);
      (void)hipEventRecord(ev[2 * r + 1], s->stream);
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) st = fail(FOE_EDEVICE, "trial launches failed");
    for (int r = 0; r < reps && st == FOE_OK; ++r) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
      total += ms;
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  std::copy(saved.begin(), saved.end(), s->st_host);
  foe_status e2 = push_states(s);
  HIP_OR(hipStreamSynchronize(s->stream));
  if (st == FOE_OK && e2 == FOE_OK) *ms_mean = total / reps;
  return st != FOE_OK ? st : e2;
}

foe_status foe_autotune(foe_solver* s, const float* d_f, int32_t reps, int32_t* chosen) {
  if (!s || !d_f || reps < 1) return fail(FOE_EINVAL, "bad argument");
  const char* cache = std::getenv("FOE_TUNE_CACHE");
  const std::string key = tune_key(s);
  int best = -1;
  if (cache) {
    std::ifstream in(cache);
    std::string k;
    int c;
    while (in >> k >> c)
      if (k == key && c >= 0 && c < N_TILE_CFGS && cfg_ok(c, s->pb.engine)) best = c;
  }
  if (best < 0) {
    bool bad = false;
    foe_status st = init_from_f(s, d_f, nullptr, &bad);
    if (st != FOE_OK) return st;
    if (bad) return fail(FOE_EINPUT, "f has a non-finite or non-positive pixel");
    double best_ms = 1e30;
    hipEvent_t e0, e1;
    HIP_OR(hipEventCreate(&e0));
    HIP_OR(hipEventCreate(&e1));
    for (int c = 0; c < N_TILE_CFGS; ++c) {
      if (!cfg_ok(c, s->pb.engine)) continue;
      build_tiles(s, c);
      st = upload_tiles(s);
      if (st != FOE_OK) return st;
      // gradient at x^0, then `reps` identical trials from the same state
      launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
      launch_fused(s, fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr), s->stream);
      HIP_OR(hipEventRecord(e0, s->stream));
      for (int r = 0; r < reps; ++r) launch_fused(s, fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr), s->stream);
      HIP_OR(hipEventRecord(e1, s->stream));
      HIP_OR(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OR(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (cache) {
      std::ofstream o(cache, std::ios::app);
      o << key << " " << best << "\n";
    }
  }
  drop_graphs(s);
  build_tiles(s, best);
  foe_status st = upload_tiles(s);
  if (st != FOE_OK) return st;
  if (chosen) *chosen = best;
  return FOE_OK;
}

foe_status foe_set_tile_config(foe_solver* s, int32_t cfg) {
  if (!s || cfg < 0 || cfg >= N_TILE_CFGS) return fail(FOE_EINVAL, "bad tile configuration");
  if (!cfg_ok(cfg, s->pb.engine)) return fail(FOE_EINVAL, "the BF16 engine takes 32 x 32 and 32 x 16 tiles only");
  HIP_OR(hipStreamSynchronize(s->stream));
  drop_graphs(s);
  build_tiles(s, cfg);
  return upload_tiles(s);
}

}  // extern "C"

// ---- The allocation-free solve.  Its device workspace is one file-scope array that every call on a GPU
// shares; each GPU holds its own copy (at its own address, found once per device with
// hipGetSymbolAddress).  The name of the array is a host-side stand-in: host code uses only the address.
namespace {

constexpr size_t NOALLOC_BYTES = (size_t)24 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
__device__ __align__(256) unsigned char noalloc_scratch[NOALLOC_BYTES];
void* g_noalloc_base[NOALLOC_MAX_DEVICES] = {};
std::mutex g_noalloc_mu;
std::mutex g_noalloc_call_mu;
TapTables g_noalloc_tabs;   // host tap tables of the current call (static: no heap, no large stack frame)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte offsets of the buffers of a one-image solve inside the workspace (32 x 32 tiles).
struct NoallocLayout {
  size_t xr[3], gr[2], partials, partials2, stats, st, st2, images, tiles, kf, ka, kf16, kb16, theta, total;
};

NoallocLayout noalloc_layout(size_t n, int ntiles, int stats_rows) {
  NoallocLayout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += align256(bytes); return at; };
  for (auto& x : l.xr) x = take(sizeof(float) * n);
  for (auto& g : l.gr) g = take(sizeof(float) * n);
  l.partials = take(sizeof(double) * PART_COLS * (size_t)ntiles);
  l.partials2 = take(sizeof(double) * PART_COLS * (size_t)ntiles);
  l.stats = take(sizeof(double) * STAT_COLS * (size_t)stats_rows);
  l.st = take(sizeof(DevState));
  l.st2 = take(sizeof(DevState));
  l.images = take(sizeof(ImageDesc));
  l.tiles = take(sizeof(TileDesc) * (size_t)ntiles);
  l.kf = take(sizeof(float) * MAX_NF * KK);
  l.ka = take(sizeof(float) * MAX_NF * KK);
  l.kf16 = take(sizeof(unsigned) * (MAX_NF / V_NC) * F16_OPS);
  l.kb16 = take(sizeof(unsigned) * MAX_NF * KB16_W);
  l.theta = take(sizeof(float) * MAX_NF);
  l.total = o;
  return l;
}

// The workspace address on the current device, looked up on the first call there.
foe_status noalloc_base(void** out) {
  int dev = -1;
  HIP_OR(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(FOE_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_base[dev]) {
    void* ptr = nullptr;
    HIP_OR(hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)));
    if (!ptr) return fail(FOE_EDEVICE, "hipGetSymbolAddress returned NULL for the workspace");
    g_noalloc_base[dev] = ptr;
  }
  *out = g_noalloc_base[dev];
  return FOE_OK;
}

// The iteration loop of run_loop for one image with direct launches in place of the graphs: the same
// kernels with the same arguments in the same order, so the results are the same bits.  Host state lives in
// s->st_host (caller memory); nothing is allocated.
foe_status run_loop_direct(foe_solver* s, int iters, foe_summary* sum, double* stats_host) {
  const double L0 = s->p.L0;
  reset_states(s, &L0, iters);
  foe_status e = push_states(s);
  if (e != FOE_OK) return e;
  launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
  launch_decide(s, DECIDE_INIT, s->stream);
  HIP_OR(hipGetLastError());
  e = pull_states(s);
  if (e != FOE_OK) return e;
  const double G0 = s->st_host[0].sums[1];
  for (;;) {
    const DevState& h = s->st_host[0];
    const int remaining = h.done ? 0 : h.target - h.iter;
    if (remaining <= 0) break;
    int q = 0;
    for (int k = 0; k < remaining; ++k) {
      FusedArgs a = fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr);
      a.decide_prev = 1;
      a.st = q ? s->st2 : s->st;
      a.st_out = q ? s->st : s->st2;
      a.part_in = q ? s->partials2 : s->partials;
      a.partials = q ? s->partials : s->partials2;
      launch_fused(s, a, s->stream);
      q ^= 1;
    }
    launch_decide(s, DECIDE_STEP, s->stream, q);
    if (q) HIP_OR(hipMemcpyAsync(s->st, s->st2, sizeof(DevState), hipMemcpyDeviceToDevice, s->stream));
    HIP_OR(hipGetLastError());
    e = pull_states(s);
    if (e != FOE_OK) return e;
  }
  const DevState& h = s->st_host[0];
  double last[STAT_COLS] = {};
  if (h.iter > 0) {
    if (stats_host) {
      HIP_OR(hipMemcpy(stats_host, s->stats, sizeof(double) * STAT_COLS * h.iter, hipMemcpyDeviceToHost));
      std::memcpy(last, stats_host + (size_t)(h.iter - 1) * STAT_COLS, sizeof(last));
    } else {
      HIP_OR(hipMemcpy(last, s->stats + (size_t)(h.iter - 1) * STAT_COLS, sizeof(last), hipMemcpyDeviceToHost));
    }
  }
  if (sum) {
    sum->iters_done = h.iter;
    sum->total_trials = h.total_trials;
    sum->F = h.Fcur;
    sum->G = h.iter > 0 ? last[1] : G0;
    sum->alpha = h.iter > 0 ? last[3] : h.alpha;
    sum->H = sum->F + sum->G;
    sum->L = h.L_acc;
  }
  return h.status != ST_OK ? status_of(h.status) : FOE_OK;
}

}  // namespace

extern "C" {

foe_status foe_solve_noalloc(const foe_params* p, const float* filters_host, const float* weights_host,
                             void* hip_stream, const float* d_f, const float* d_init, float* d_u_out,
                             foe_summary* sum_host, double* stats_host) {
  if (!p || !d_f || !d_u_out) return fail(FOE_EINVAL, "NULL argument");
  Problem pb;
  foe_status v = validate(p, filters_host, weights_host, &pb);
  if (v != FOE_OK) return v;
  if (p->fusion != FOE_FUSED) return fail(FOE_EINVAL, "the allocation-free solve runs the fused kernel only");
  ImageDesc im{};
  v = image_desc(p, p->height, p->width, p->lambda1, p->lambda2, p->looks, &im);
  if (v != FOE_OK) return v;
  const TileCfg tc = TILE_CFGS[0];
  const int ntx = (p->width + tc.tw - 1) / tc.tw, nty = (p->height + tc.th - 1) / tc.th;
  const size_t n = (size_t)p->height * p->width;
  const int stats_rows = p->max_iters > 0 ? p->max_iters : 1;
  if ((int64_t)ntx * nty > (int64_t)1 << 24) return fail(FOE_EINVAL, "image too large for the allocation-free solve");
  const int ntiles = ntx * nty;
  const NoallocLayout l = noalloc_layout(n, ntiles, stats_rows);
  if (l.total > NOALLOC_BYTES)
    return fail(FOE_EINVAL, "the allocation-free solve holds " + std::to_string(NOALLOC_BYTES) +
                                " bytes of device workspace; this image and max_iters need " + std::to_string(l.total));
  im.off = 0;
  im.tile0 = 0;
  im.ntiles = ntiles;
  void* base = nullptr;
  v = noalloc_base(&base);
  if (v != FOE_OK) return v;
  unsigned char* b = static_cast<unsigned char*>(base);

  // one call at a time per process: the host tap tables are static, and calls that overlap on a GPU race
  // on its workspace anyway
  std::lock_guard<std::mutex> lock(g_noalloc_call_mu);
  foe_solver s;   // its containers stay empty: nothing here allocates
  DevState st_host{};
  TapTables& tabs = g_noalloc_tabs;
  s.p = *p;
  s.pb = pb;
  s.stream = (hipStream_t)hip_stream;
  s.n_img = 1;
  s.n = n;
  s.tile_cfg = 0;
  s.nblocks = ntiles;
  s.max_tiles = ntiles;
  for (int i = 0; i < 3; ++i) s.xr[i] = reinterpret_cast<float*>(b + l.xr[i]);
  for (int i = 0; i < 2; ++i) s.gr[i] = reinterpret_cast<float*>(b + l.gr[i]);
  s.fbuf = const_cast<float*>(d_f);   // f is only read
  s.partials = reinterpret_cast<double*>(b + l.partials);
  s.partials2 = reinterpret_cast<double*>(b + l.partials2);
  s.stats = reinterpret_cast<double*>(b + l.stats);
  s.stats_rows = stats_rows;
  s.st = reinterpret_cast<DevState*>(b + l.st);
  s.st2 = reinterpret_cast<DevState*>(b + l.st2);
  s.st_host = &st_host;
  s.d_images = reinterpret_cast<ImageDesc*>(b + l.images);
  s.d_tiles = reinterpret_cast<TileDesc*>(b + l.tiles);
  s.kf = reinterpret_cast<float*>(b + l.kf);
  s.ka = reinterpret_cast<float*>(b + l.ka);
  s.kf16 = reinterpret_cast<unsigned*>(b + l.kf16);
  s.kb16 = reinterpret_cast<unsigned*>(b + l.kb16);
  s.theta = reinterpret_cast<float*>(b + l.theta);

  build_tap_tables(p->num_filters, filters_host, weights_host, &tabs);
  HIP_OR(hipMemcpyAsync(s.kf, tabs.kf, sizeof(tabs.kf), hipMemcpyHostToDevice, s.stream));
  HIP_OR(hipMemcpyAsync(s.ka, tabs.ka, sizeof(tabs.ka), hipMemcpyHostToDevice, s.stream));
  HIP_OR(hipMemcpyAsync(s.kf16, tabs.kf16, sizeof(tabs.kf16), hipMemcpyHostToDevice, s.stream));
  HIP_OR(hipMemcpyAsync(s.kb16, tabs.kb16, sizeof(tabs.kb16), hipMemcpyHostToDevice, s.stream));
  HIP_OR(hipMemcpyAsync(s.theta, tabs.theta, sizeof(tabs.theta), hipMemcpyHostToDevice, s.stream));
  HIP_OR(hipMemcpyAsync(s.d_images, &im, sizeof(ImageDesc), hipMemcpyHostToDevice, s.stream));
  tile_list_kernel<<<(ntiles + 255) / 256, 256, 0, s.stream>>>(s.d_tiles, ntx, ntiles, tc.tw, tc.th);
  HIP_OR(hipGetLastError());

  // a1: x^0 = x^-1 from f (or d_init), with the input check
  reset_states(&s, &s.p.L0, s.p.max_iters);
  foe_status e = push_states(&s);
  if (e != FOE_OK) return e;
  const size_t blocks = std::min<size_t>(std::max<size_t>((n + 255) / 256, 1), 1024);
  init_state_kernel<<<dim3((unsigned)blocks, 1, 1), 256, 0, s.stream>>>(s.fbuf, d_init, s.xr[0], s.xr[1], s.d_images,
                                                                        s.pb.model, s.st);
  HIP_OR(hipGetLastError());
  e = pull_states(&s);
  if (e != FOE_OK) return e;
  foe_status st;
  if (st_host.input_bad) {
    st = fail(FOE_EINPUT, "f or the initial image has a non-finite or non-positive pixel");
    if (sum_host) std::memset(sum_host, 0, sizeof(foe_summary));
  } else {
    st = run_loop_direct(&s, s.p.max_iters, sum_host, stats_host);
  }
  finalize_kernel<<<dim3((unsigned)blocks, 1, 1), 256, 0, s.stream>>>(s.st, s.xr[0], s.xr[1], s.xr[2], d_u_out,
                                                                      s.d_images, s.pb.model);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s.stream));
  return st;
}

const char* foe_status_str(foe_status st) {
  switch (st) {
    case FOE_OK: return "FOE_OK";
    case FOE_EINVAL: return "FOE_EINVAL";
    case FOE_ENOMEM: return "FOE_ENOMEM";
    case FOE_EDEVICE: return "FOE_EDEVICE";
    case FOE_ELINESEARCH: return "FOE_ELINESEARCH";
    case FOE_ENONFINITE: return "FOE_ENONFINITE";
    case FOE_EINPUT: return "FOE_EINPUT";
  }
  return "FOE_UNKNOWN";
}

const char* foe_last_error(void) { return g_last_error.c_str(); }

int32_t foe_abi_version(void) { return FOE_ABI_VERSION; }

}  // extern "C"
