// Host runtime and C ABI of the FoE + iPiano library (declared in include/foe.h).
//
// A solver owns, per image: the x ring (x^n, x^{n-1}, candidate), the gradient ring
// (grad F(x^n), candidate grad F(x+)), a copy of f, per-block partial sums, the device
// iPiano state and the stats ring.  The iteration loop is a sequence of "slots", each one
// fused trial launch followed by one single-block decide launch; the decision lives on the
// device, so the host only synchronises between rounds of slots (one round when no trial
// is rejected).  Rounds are replayed from pre-instantiated HIP graphs of 16 and 1 slots.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/foe.h"
#include "common.hpp"
#include "kernels_valu.hpp"
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

// Default tile configuration of the VALU engine.
constexpr int V_TW = 32, V_TH = 32, V_NC = 16, V_NT = 512, V_BR = 4, V_BC = 2;
constexpr int GRAPH_BIG = 16;

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

}  // namespace

struct foe_solver {
  foe_params p{};
  Problem pb{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  size_t n = 0;
  float* xr[3] = {nullptr, nullptr, nullptr};
  float* gr[2] = {nullptr, nullptr};
  float* fbuf = nullptr;
  float* scratch = nullptr;  // probe workspace (one plane)
  float* kf = nullptr;
  float* ka = nullptr;
  float* theta = nullptr;
  double* partials = nullptr;
  double* stats = nullptr;
  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned mirror
  int tiles_x = 0, tiles_y = 0, nblocks = 0;
  hipGraphExec_t graph_big = nullptr, graph_one = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int last_launches = 0;
};

namespace {

FusedArgs fused_args(foe_solver* s, int mode, const float* f, const float* x_in, float* g_out) {
  FusedArgs a;
  a.pb = s->pb;
  a.f = f;
  a.xr0 = s->xr[0]; a.xr1 = s->xr[1]; a.xr2 = s->xr[2];
  a.gr0 = s->gr[0]; a.gr1 = s->gr[1];
  a.x_in = x_in;
  a.g_out = g_out;
  a.st = s->st;
  a.partials = s->partials;
  a.kf = s->kf;
  a.ka = s->ka;
  a.theta = s->theta;
  a.tiles_x = s->tiles_x;
  a.mode = mode;
  return a;
}

void launch_fused(foe_solver* s, const FusedArgs& a, hipStream_t stream) {
  if (s->pb.engine == FWD_MFMA_BF16)
    fused_valu_kernel<V_TW, V_TH, V_NC, V_NT, V_BR, V_BC, FWD_MFMA_BF16><<<s->nblocks, V_NT, 0, stream>>>(a);
  else if (s->pb.engine == FWD_MFMA_F32)
    fused_valu_kernel<V_TW, V_TH, V_NC, V_NT, V_BR, V_BC, FWD_MFMA_F32><<<s->nblocks, V_NT, 0, stream>>>(a);
  else
    fused_valu_kernel<V_TW, V_TH, V_NC, V_NT, V_BR, V_BC, FWD_VALU><<<s->nblocks, V_NT, 0, stream>>>(a);
}

void launch_decide(foe_solver* s, int mode, hipStream_t stream) {
  decide_kernel<<<1, 256, 0, stream>>>(s->st, s->partials, s->nblocks, s->pb, s->stats, mode);
}

int grid_1d(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

foe_status validate(const foe_params* p, const float* filters, const float* weights, Problem* pb) {
  if (!p) return fail(FOE_EINVAL, "params is NULL");
  if (!filters || !weights) return fail(FOE_EINVAL, "filters/weights is NULL");
  if (p->height < 4 || p->width < 4) return fail(FOE_EINVAL, "height and width must be >= 4");
  if ((int64_t)p->height * p->width > ((int64_t)1 << 31)) return fail(FOE_EINVAL, "image too large");
  if (p->num_filters < 1 || p->num_filters > FOE_MAX_FILTERS) return fail(FOE_EINVAL, "num_filters out of range");
  if (p->ksize != FOE_KSIZE) return fail(FOE_EINVAL, "ksize must be 7");
  if (p->model < 0 || p->model > 2) return fail(FOE_EINVAL, "bad model");
  if (p->boundary < 0 || p->boundary > 2) return fail(FOE_EINVAL, "bad boundary");
  if (p->precision != FOE_PREC_FP32 && p->precision != FOE_PREC_BF16) return fail(FOE_EINVAL, "bad precision");
  if (p->precision == FOE_PREC_BF16 && p->engine == FOE_ENGINE_VALU)
    return fail(FOE_EINVAL, "BF16 precision runs on the MFMA engine");
  if (p->engine < FOE_ENGINE_AUTO || p->engine > FOE_ENGINE_MFMA) return fail(FOE_EINVAL, "bad engine");
  if (p->step_mode != FOE_STEP_BACKTRACK && p->step_mode != FOE_STEP_FIXED) return fail(FOE_EINVAL, "bad step_mode");
  if (p->looks < 1) return fail(FOE_EINVAL, "looks must be >= 1");
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
  double l1 = p->lambda1, l2 = p->lambda2;
  if (p->model == FOE_MODEL_IDIV) {
    if (!(std::isfinite(l1) && l1 >= 0.0)) return fail(FOE_EINVAL, "IDIV needs lambda1 >= 0");
  } else {
    double d1, d2;
    paper_lambdas(p->looks, &d1, &d2);
    if (l1 < 0.0) l1 = d1;
    if (l2 < 0.0) l2 = d2;
    if (!std::isfinite(l1) || !std::isfinite(l2)) return fail(FOE_EINVAL, "lambda must be finite");
  }
  if (p->model == FOE_MODEL_LOG) l2 = 0.0;
  for (int i = 0; i < p->num_filters * FOE_KSIZE * FOE_KSIZE; ++i)
    if (!std::isfinite(filters[i])) return fail(FOE_EINVAL, "non-finite filter tap");
  for (int i = 0; i < p->num_filters; ++i)
    if (!(std::isfinite(weights[i]) && weights[i] >= 0.0f)) return fail(FOE_EINVAL, "weights must be finite, >= 0");
  pb->H = p->height;
  pb->W = p->width;
  pb->nf = p->num_filters;
  pb->model = p->model;
  pb->bc = p->boundary;
  pb->step_mode = p->step_mode;
  pb->max_backtracks = p->max_backtracks;
  pb->newton_iters = p->newton_iters;
  pb->lam1 = (float)l1;
  pb->lam2 = (float)l2;
  pb->beta = (float)p->beta;
  pb->beta_d = p->beta;
  pb->eta_up = p->eta_up;
  pb->eta_down = p->eta_down;
  pb->alpha_fixed = p->alpha_fixed;
  pb->engine = p->precision == FOE_PREC_BF16 ? FWD_MFMA_BF16
               : (p->engine == FOE_ENGINE_VALU ? FWD_VALU : FWD_MFMA_F32);
  return FOE_OK;
}

void destroy_all(foe_solver* s) {
  if (!s) return;
  if (s->graph_big) (void)hipGraphExecDestroy(s->graph_big);
  if (s->graph_one) (void)hipGraphExecDestroy(s->graph_one);
  for (float* p : s->xr) if (p) (void)hipFree(p);
  for (float* p : s->gr) if (p) (void)hipFree(p);
  if (s->fbuf) (void)hipFree(s->fbuf);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->kf) (void)hipFree(s->kf);
  if (s->ka) (void)hipFree(s->ka);
  if (s->theta) (void)hipFree(s->theta);
  if (s->partials) (void)hipFree(s->partials);
  if (s->stats) (void)hipFree(s->stats);
  if (s->st) (void)hipFree(s->st);
  if (s->st_host) (void)hipHostFree(s->st_host);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  delete s;
}

foe_status build_graph(foe_solver* s, int slots, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_OR(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
  FusedArgs a = fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr);
  for (int k = 0; k < slots; ++k) {
    launch_fused(s, a, s->cap_stream);
    launch_decide(s, DECIDE_STEP, s->cap_stream);
  }
  HIP_OR(hipStreamEndCapture(s->cap_stream, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(FOE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return FOE_OK;
}

// Host-side initial device state for a launch sequence of `iters` iterations from ring slots 0/1.
void reset_state(foe_solver* s, double L_in, int iters) {
  DevState& h = *s->st_host;
  std::memset(&h, 0, sizeof(DevState));
  h.icur = 0; h.iprev = 1; h.icand = 2;
  h.gcur = 0; h.gcand = 1;
  h.target = iters;
  if (s->pb.step_mode == FIXED) {
    h.L = L_in;
    h.alpha = s->pb.alpha_fixed;
  } else {
    h.L = s->pb.eta_down * L_in;
    h.alpha = 1.9 * (1.0 - s->pb.beta_d) / h.L;
  }
  h.L_acc = L_in;
}

// Runs the iteration loop from ring slots 0 (x^n) and 1 (x^{n-1}); fbuf holds f.
foe_status run_loop(foe_solver* s, double L_in, int iters, foe_summary* sum, double* stats_host) {
  reset_state(s, L_in, iters);
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
  // F, G and grad F at x^0
  launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
  launch_decide(s, DECIDE_INIT, s->stream);
  HIP_OR(hipGetLastError());
  if (!s->graph_big) {
    foe_status e = build_graph(s, GRAPH_BIG, &s->graph_big);
    if (e != FOE_OK) return e;
    e = build_graph(s, 1, &s->graph_one);
    if (e != FOE_OK) return e;
  }
  HIP_OR(hipEventRecord(s->ev0, s->stream));
  int remaining = iters;
  int launches = 0;
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  double G0 = s->st_host->sums[1];
  while (remaining > 0 && !s->st_host->done) {
    for (int k = 0; k < remaining / GRAPH_BIG; ++k) HIP_OR(hipGraphLaunch(s->graph_big, s->stream));
    for (int k = 0; k < remaining % GRAPH_BIG; ++k) HIP_OR(hipGraphLaunch(s->graph_one, s->stream));
    launches += remaining;
    HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    HIP_OR(hipStreamSynchronize(s->stream));
    remaining = s->st_host->target - s->st_host->iter;
  }
  HIP_OR(hipEventRecord(s->ev1, s->stream));
  HIP_OR(hipEventSynchronize(s->ev1));
  float ms = 0.f;
  HIP_OR(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  s->last_ms = ms;
  s->last_launches = launches;
  const DevState& h = *s->st_host;
  if (stats_host && h.iter > 0)
    HIP_OR(hipMemcpy(stats_host, s->stats, sizeof(double) * STAT_COLS * h.iter, hipMemcpyDeviceToHost));
  if (sum) {
    sum->iters_done = h.iter;
    sum->total_trials = h.total_trials;
    sum->F = h.Fcur;
    if (h.iter > 0) {
      double row[STAT_COLS];
      HIP_OR(hipMemcpy(row, s->stats + (size_t)(h.iter - 1) * STAT_COLS, sizeof(row), hipMemcpyDeviceToHost));
      sum->G = row[1];
      sum->alpha = row[3];
    } else {
      sum->G = G0;
      sum->alpha = h.alpha;
    }
    sum->H = sum->F + sum->G;
    sum->L = h.L_acc;
  }
  switch (h.status) {
    case ST_OK: return FOE_OK;
    case ST_ELINESEARCH: return fail(FOE_ELINESEARCH, "backtracking exceeded max_backtracks");
    case ST_ENONFINITE: return fail(FOE_ENONFINITE, "non-finite energy or reduction");
    case ST_EINPUT: return fail(FOE_EINPUT, "f or the initial image has a non-finite or non-positive pixel");
    default: return fail(FOE_EDEVICE, "unknown device status");
  }
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
  if (!out) return fail(FOE_EINVAL, "out is NULL");
  Problem pb;
  foe_status v = validate(p, filters_host, weights_host, &pb);
  if (v != FOE_OK) return v;
  foe_solver* s = new (std::nothrow) foe_solver();
  if (!s) return fail(FOE_ENOMEM, "host allocation failed");
  s->p = *p;
  s->pb = pb;
  s->stream = (hipStream_t)hip_stream;
  s->n = (size_t)p->height * p->width;
  s->tiles_x = (p->width + V_TW - 1) / V_TW;
  s->tiles_y = (p->height + V_TH - 1) / V_TH;
  s->nblocks = s->tiles_x * s->tiles_y;
  const size_t plane = sizeof(float) * s->n;
  auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
  bool ok = true;
  for (auto& x : s->xr) ok = ok && alloc((void**)&x, plane);
  for (auto& g : s->gr) ok = ok && alloc((void**)&g, plane);
  ok = ok && alloc((void**)&s->fbuf, plane) && alloc((void**)&s->scratch, plane);
  ok = ok && alloc((void**)&s->kf, sizeof(float) * MAX_NF * KK) && alloc((void**)&s->ka, sizeof(float) * MAX_NF * KK);
  ok = ok && alloc((void**)&s->theta, sizeof(float) * MAX_NF);
  ok = ok && alloc((void**)&s->partials, sizeof(double) * PART_COLS * (size_t)s->nblocks);
  ok = ok && alloc((void**)&s->stats, sizeof(double) * STAT_COLS * (size_t)(p->max_iters > 0 ? p->max_iters : 1));
  ok = ok && alloc((void**)&s->st, sizeof(DevState));
  ok = ok && hipHostMalloc((void**)&s->st_host, sizeof(DevState), hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    destroy_all(s);
    return fail(FOE_ENOMEM, "device allocation failed");
  }
  std::vector<float> kf(MAX_NF * KK, 0.0f), ka(MAX_NF * KK, 0.0f), th(MAX_NF, 0.0f);
  for (int i = 0; i < p->num_filters; ++i) {
    th[i] = weights_host[i];
    for (int a = 0; a < KS; ++a)
      for (int b = 0; b < KS; ++b) {
        float k = filters_host[(size_t)i * KK + a * KS + b];
        ka[i * KK + a * KS + b] = k;
        const int c = i / V_NC, j = i % V_NC, t = (KS - 1 - a) * KS + (KS - 1 - b);
        kf[((size_t)c * KK + t) * V_NC + j] = k;
      }
  }
  hipError_t e = hipMemcpy(s->kf, kf.data(), sizeof(float) * kf.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->ka, ka.data(), sizeof(float) * ka.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->theta, th.data(), sizeof(float) * th.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&s->ev0);
  if (e == hipSuccess) e = hipEventCreate(&s->ev1);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    destroy_all(s);
    return fail(FOE_EDEVICE, std::string("foe_create: ") + hipGetErrorString(e));
  }
  *out = s;
  return FOE_OK;
}

foe_status foe_destroy(foe_solver* s) {
  if (!s) return fail(FOE_EINVAL, "solver is NULL");
  (void)hipStreamSynchronize(s->stream);
  destroy_all(s);
  return FOE_OK;
}

foe_status foe_solve(foe_solver* s, const float* d_f, const float* d_init, float* d_u_out, foe_summary* sum_host,
                     double* stats_host) {
  if (!s || !d_f || !d_u_out) return fail(FOE_EINVAL, "NULL argument");
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  reset_state(s, s->p.L0, s->p.max_iters);  // ring slot 0 = x^0 even if the input is rejected
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
  init_state_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(s->fbuf, d_init, s->xr[0], s->xr[1], s->n, s->pb.model,
                                                          s->st);
  // run_loop resets the state struct; carry the input flag through it
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  const int bad = s->st_host->input_bad;
  foe_status st;
  if (bad) {
    st = fail(FOE_EINPUT, "f or the initial image has a non-finite or non-positive pixel");
    if (sum_host) std::memset(sum_host, 0, sizeof(*sum_host));
  } else {
    st = run_loop(s, s->p.L0, s->p.max_iters, sum_host, stats_host);
  }
  finalize_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(s->st, s->xr[0], s->xr[1], s->xr[2], d_u_out, s->n,
                                                        s->pb.model);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  return st;
}

foe_status foe_solve_from(foe_solver* s, const float* d_f, float* d_x_cur, float* d_x_prev, double* L_inout,
                          int32_t iters, foe_summary* sum_host, double* stats_host) {
  if (!s || !d_f || !d_x_cur || !d_x_prev || !L_inout) return fail(FOE_EINVAL, "NULL argument");
  if (iters < 0 || iters > s->p.max_iters) return fail(FOE_EINVAL, "iters must be in [0, max_iters]");
  if (!finite_pos(*L_inout)) return fail(FOE_EINVAL, "L must be > 0");
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[0], d_x_cur, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[1], d_x_prev, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemsetAsync(&s->st->input_bad, 0, sizeof(int), s->stream));
  check_input_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(s->fbuf, s->n, s->st);
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  if (s->st_host->input_bad) return fail(FOE_EINPUT, "f has a non-finite or non-positive pixel");
  foe_status st = run_loop(s, *L_inout, iters, sum_host, stats_host);
  export_state_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(s->st, s->xr[0], s->xr[1], s->xr[2], d_x_cur, d_x_prev,
                                                            s->n);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  *L_inout = s->st_host->L_acc;
  return st;
}

foe_status foe_eval_gradient(foe_solver* s, const float* d_x, float* d_grad) {
  if (!s || !d_x || !d_grad) return fail(FOE_EINVAL, "NULL argument");
  // G is not needed; f = x keeps the data-term arithmetic finite
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
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  if (F) *F = s->st_host->sums[0];
  if (G) *G = s->st_host->sums[1];
  return FOE_OK;
}

foe_status foe_eval_prox(foe_solver* s, const float* d_xhat, const float* d_f, double tau, float* d_out) {
  if (!s || !d_xhat || !d_f || !d_out) return fail(FOE_EINVAL, "NULL argument");
  if (!finite_pos(tau)) return fail(FOE_EINVAL, "tau must be > 0");
  prox_probe_kernel<<<grid_1d(s->n), 256, 0, s->stream>>>(d_xhat, d_f, d_out, s->n, (float)tau, s->pb);
  HIP_OR(hipGetLastError());
  HIP_OR(hipStreamSynchronize(s->stream));
  return FOE_OK;
}

foe_status foe_step(foe_solver* s, const float* d_f, const float* d_x, const float* d_xprev, double L_forced,
                    float* d_xnext, double* info_host) {
  if (!s || !d_f || !d_x || !d_xprev || !d_xnext) return fail(FOE_EINVAL, "NULL argument");
  if (s->pb.step_mode == BACKTRACK && !finite_pos(L_forced)) return fail(FOE_EINVAL, "L_forced must be > 0");
  // ring: slot 0 = x, slot 1 = xprev, slot 2 = output; gradient of x into gr[0]
  HIP_OR(hipMemcpyAsync(s->fbuf, d_f, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[0], d_x, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->xr[1], d_xprev, sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  launch_fused(s, fused_args(s, MODE_EVAL, s->fbuf, s->xr[0], s->gr[0]), s->stream);
  DevState& h = *s->st_host;
  std::memset(&h, 0, sizeof(DevState));
  h.icur = 0; h.iprev = 1; h.icand = 2; h.gcur = 0; h.gcand = 1; h.target = 1;
  h.L = L_forced;
  h.alpha = s->pb.step_mode == FIXED ? s->pb.alpha_fixed : 1.9 * (1.0 - s->pb.beta_d) / L_forced;
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
  launch_fused(s, fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr), s->stream);
  launch_decide(s, DECIDE_REPORT, s->stream);
  HIP_OR(hipGetLastError());
  HIP_OR(hipMemcpyAsync(d_xnext, s->xr[2], sizeof(float) * s->n, hipMemcpyDeviceToDevice, s->stream));
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
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

foe_status foe_profile_trial(foe_solver* s, int32_t reps, double* ms_mean) {
  if (!s || reps < 1 || !ms_mean) return fail(FOE_EINVAL, "bad argument");
  if (!s->graph_big) return fail(FOE_EINVAL, "run foe_solve first");
  HIP_OR(hipMemcpyAsync(s->st_host, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  DevState saved = *s->st_host;
  s->st_host->done = 0;
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  foe_status status = FOE_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) status = fail(FOE_EDEVICE, "hipEventCreate failed");
  const FusedArgs a = fused_args(s, MODE_TRIAL, s->fbuf, nullptr, nullptr);
  double total = 0.0;
  if (status == FOE_OK) {
    for (int r = 0; r < reps; ++r) {
      (void)hipEventRecord(ev[2 * r], s->stream);
      launch_fused(s, a, s->stream);
      (void)hipEventRecord(ev[2 * r + 1], s->stream);
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) status = fail(FOE_EDEVICE, "trial launches failed");
    for (int r = 0; r < reps && status == FOE_OK; ++r) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]);
      total += ms;
    }
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  *s->st_host = saved;
  HIP_OR(hipMemcpyAsync(s->st, s->st_host, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
  HIP_OR(hipStreamSynchronize(s->stream));
  if (status == FOE_OK) *ms_mean = total / reps;
  return status;
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
