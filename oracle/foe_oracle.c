/*
 * FP64 CPU oracle of the FoE + iPiano despeckling model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or table with the HIP library.
 *
 * Plain, slow, obviously correct: every quantity is computed in double from
 * its definition in the paper, in the order the paper states it.
 *
 *   FoE prior            E_FoE(u) = sum_i theta_i sum_p rho((k_i * u)_p)     Sec. II-A, eq. (FOEmodel)
 *   Lorentzian           rho(x) = log(1 + x^2), rho'(x) = 2x / (1 + x^2)      Sec. II-A, Sec. II-C
 *   log model            F(w) = E_FoE(e^w), G(w) = lam/2 <2w + f^2 e^{-2w}, 1> Sec. II-C, eq. (original)
 *   combined model       G(w) = lam1/2 (2w + f^2 e^{-2w}) + lam2/2 (e^{2w} - 2 f^2 w)   Sec. III-A, eq. (newmodel)
 *   I-divergence model   F(u) = E_FoE(u), G(u) = lam/2 <u^2 - 2 f^2 log u, 1>  Sec. II-B, eq. (variant)
 *   gradients            grad_w F = sum_i theta_i W K_i^T rho'(K_i e^w), W = diag(e^w);
 *                        grad_u F = sum_i theta_i K_i^T rho'(K_i u)              Sec. II-C
 *   prox                 (I + tau dG)^{-1}: Newton for the log / combined model,
 *                        the closed-form root for the I-divergence model       Sec. II-C, eq. (subproblem)
 *   iPiano               u+ = (I + a dG)^{-1}(u - a grad F(u) + b (u - u_prev))  Sec. II-C, eq. (fplusg)
 *
 * K_i is the convolution of the image with k_i (true convolution, centre tap
 * (3,3)) applied to the image extended by a 3-pixel boundary map P:
 *   K_i x = C_i P x,   K_i^T v = P^T C_i^T v.
 * The paper does not state the boundary; SYMMETRIC (half-sample reflection),
 * ZERO and PERIODIC are provided.  The backtracking rule for the step (accept
 * when F(x+) <= F(x) + <grad F(x), d> + L/2 |d|^2, else L <- eta_up L) is the
 * descent-lemma test iPiano's Lipschitz estimate is built on.
 *
 * Sums that reduce an image to a scalar are taken per row, then over rows in
 * increasing row order, so results do not depend on the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_K 7
#define ORA_R 3

enum { ORA_COMBINED = 0, ORA_LOG = 1, ORA_IDIV = 2 };
enum { ORA_SYMMETRIC = 0, ORA_ZERO = 1, ORA_PERIODIC = 2 };
enum { ORA_BACKTRACK = 0, ORA_FIXED = 1 };
enum { ORA_OK = 0, ORA_EINVAL = 1, ORA_ENOMEM = 2, ORA_ELINESEARCH = 4, ORA_ENONFINITE = 5, ORA_EINPUT = 6 };

typedef struct {
  int32_t model, boundary, step_mode, max_backtracks;
  double lam1, lam2, beta, alpha_fixed, eta_up, eta_down;
} ora_params;

void ora_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int ora_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Boundary map P: index q of the extended signal (q in [-3, n+3)) -> source
 * pixel, or -1 where the extension is zero. */
static int src_index(int q, int n, int bc) {
  if (q >= 0 && q < n) return q;
  if (bc == ORA_SYMMETRIC) {
    /* half-sample mirror, repeated for sides below the filter radius: period 2n */
    int m = ((q % (2 * n)) + 2 * n) % (2 * n);
    return m < n ? m : 2 * n - 1 - m;
  }
  if (bc == ORA_PERIODIC) return ((q % n) + n) % n;
  return -1;
}

/* y = K x = C P x for one 7x7 filter:
 * y(p) = sum_{a,b} k[a][b] * (P x)(p_y + 3 - a, p_x + 3 - b). */
void ora_forward(const double* x, int H, int W, const double* k, int bc, double* y) {
#pragma omp parallel for schedule(static)
  for (int py = 0; py < H; ++py) {
    for (int px = 0; px < W; ++px) {
      double s = 0.0;
      for (int a = 0; a < ORA_K; ++a) {
        int sy = src_index(py + ORA_R - a, H, bc);
        if (sy < 0) continue;
        for (int b = 0; b < ORA_K; ++b) {
          int sx = src_index(px + ORA_R - b, W, bc);
          if (sx < 0) continue;
          s += k[a * ORA_K + b] * x[(size_t)sy * W + sx];
        }
      }
      y[(size_t)py * W + px] = s;
    }
  }
}

/* C^T v into the extended (H+6) x (W+6) domain, accumulated into ext:
 * (C^T v)(q) = sum_{a,b} k[a][b] v(q_y - 3 + a, q_x - 3 + b), v = 0 off the image.
 * This is the transpose of the valid convolution C written as a gather. */
static void ext_correlate_acc(const double* v, int H, int W, const double* k, double* ext) {
  const int We = W + 2 * ORA_R;
#pragma omp parallel for schedule(static)
  for (int ey = 0; ey < H + 2 * ORA_R; ++ey) {
    int qy = ey - ORA_R;
    for (int ex = 0; ex < We; ++ex) {
      int qx = ex - ORA_R;
      double s = 0.0;
      for (int a = 0; a < ORA_K; ++a) {
        int vy = qy - ORA_R + a;
        if (vy < 0 || vy >= H) continue;
        for (int b = 0; b < ORA_K; ++b) {
          int vx = qx - ORA_R + b;
          if (vx < 0 || vx >= W) continue;
          s += k[a * ORA_K + b] * v[(size_t)vy * W + vx];
        }
      }
      ext[(size_t)ey * We + ex] += s;
    }
  }
}

/* out = P^T ext: every extended sample is added onto the pixel it was copied from. */
static void fold(const double* ext, int H, int W, int bc, double* out) {
  const int We = W + 2 * ORA_R;
  memset(out, 0, sizeof(double) * (size_t)H * W);
  /* serial: several extended samples may land on one pixel */
  for (int ey = 0; ey < H + 2 * ORA_R; ++ey) {
    int sy = src_index(ey - ORA_R, H, bc);
    if (sy < 0) continue;
    for (int ex = 0; ex < We; ++ex) {
      int sx = src_index(ex - ORA_R, W, bc);
      if (sx < 0) continue;
      out[(size_t)sy * W + sx] += ext[(size_t)ey * We + ex];
    }
  }
}

/* out = K^T v = P^T C^T v for one filter. */
int ora_adjoint(const double* v, int H, int W, const double* k, int bc, double* out) {
  size_t ne = (size_t)(H + 2 * ORA_R) * (W + 2 * ORA_R);
  double* ext = (double*)calloc(ne, sizeof(double));
  if (!ext) return ORA_ENOMEM;
  ext_correlate_acc(v, H, W, k, ext);
  fold(ext, H, W, bc, out);
  free(ext);
  return ORA_OK;
}

static int uses_log(int model) { return model == ORA_COMBINED || model == ORA_LOG; }

/* u(x): the amplitude the FoE prior acts on (e^w for the log models, u itself otherwise). */
static void amplitude(const double* x, size_t n, int model, double* u) {
  for (size_t p = 0; p < n; ++p) u[p] = uses_log(model) ? exp(x[p]) : x[p];
}

static double sum_rows(const double* e, int H, int W) {
  double* rows = (double*)malloc(sizeof(double) * (size_t)H);
  if (!rows) return NAN;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < H; ++y) {
    double s = 0.0;
    for (int x = 0; x < W; ++x) s += e[(size_t)y * W + x];
    rows[y] = s;
  }
  double t = 0.0;
  for (int y = 0; y < H; ++y) t += rows[y];
  free(rows);
  return t;
}

/* F(x) = sum_i theta_i sum_p log(1 + (K_i u(x))_p^2). */
double ora_energy_F(const double* x, int H, int W, const double* bank, const double* theta, int nf, int model,
                    int bc) {
  size_t n = (size_t)H * W;
  double* u = (double*)malloc(sizeof(double) * n);
  double* y = (double*)malloc(sizeof(double) * n);
  double* e = (double*)calloc(n, sizeof(double));
  if (!u || !y || !e) { free(u); free(y); free(e); return NAN; }
  amplitude(x, n, model, u);
  for (int i = 0; i < nf; ++i) {
    ora_forward(u, H, W, bank + (size_t)i * ORA_K * ORA_K, bc, y);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)n; ++p) e[p] += theta[i] * log1p(y[p] * y[p]);
  }
  double F = sum_rows(e, H, W);
  free(u); free(y); free(e);
  return F;
}

/* Per-pixel data term g(x_p; f_p). */
static double data_term(double x, double f, int model, double lam1, double lam2) {
  double f2 = f * f;
  if (model == ORA_IDIV) return 0.5 * lam1 * (x * x - 2.0 * f2 * log(x));
  double t = 0.5 * lam1 * (2.0 * x + f2 * exp(-2.0 * x));
  if (model == ORA_COMBINED) t += 0.5 * lam2 * (exp(2.0 * x) - 2.0 * f2 * x);
  return t;
}

double ora_energy_G(const double* x, const double* f, int H, int W, int model, double lam1, double lam2) {
  size_t n = (size_t)H * W;
  double* e = (double*)malloc(sizeof(double) * n);
  if (!e) return NAN;
#pragma omp parallel for schedule(static)
  for (long p = 0; p < (long)n; ++p) e[p] = data_term(x[p], f[p], model, lam1, lam2);
  double G = sum_rows(e, H, W);
  free(e);
  return G;
}

/* grad F(x) = [u(x) .*] sum_i theta_i K_i^T rho'(K_i u(x)). */
int ora_grad_F(const double* x, int H, int W, const double* bank, const double* theta, int nf, int model, int bc,
               double* grad) {
  size_t n = (size_t)H * W;
  size_t ne = (size_t)(H + 2 * ORA_R) * (W + 2 * ORA_R);
  double* u = (double*)malloc(sizeof(double) * n);
  double* y = (double*)malloc(sizeof(double) * n);
  double* ext = (double*)calloc(ne, sizeof(double));
  if (!u || !y || !ext) { free(u); free(y); free(ext); return ORA_ENOMEM; }
  amplitude(x, n, model, u);
  for (int i = 0; i < nf; ++i) {
    const double* k = bank + (size_t)i * ORA_K * ORA_K;
    ora_forward(u, H, W, k, bc, y);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < (long)n; ++p) y[p] = theta[i] * 2.0 * y[p] / (1.0 + y[p] * y[p]);
    ext_correlate_acc(y, H, W, k, ext); /* sum_i C_i^T z_i; P^T is linear, applied once below */
  }
  fold(ext, H, W, bc, grad);
  if (uses_log(model))
    for (size_t p = 0; p < n; ++p) grad[p] *= u[p]; /* chain rule: W = diag(e^w) */
  free(u); free(y); free(ext);
  return ORA_OK;
}

/* prox of tau*G at one pixel.
 * Log / combined models: the root of
 *   phi(w) = w - what + tau lam1 (1 - f^2 e^{-2w}) + tau lam2 (e^{2w} - f^2),
 * which is strictly increasing; both data terms are minimised at w = log f, so
 * the root lies between what and log f.  Newton from what, with a bisection step
 * whenever an iterate leaves the bracket, to |dw| <= 1e-15 max(1, |w|).
 * I-divergence model: the positive root of (1 + tau lam) u^2 - uhat u - tau lam f^2 = 0,
 * written without cancellation for uhat < 0.  Returns the Newton iteration count. */
static int prox_pixel(double xh, double f, int model, double tau, double lam1, double lam2, double* out) {
  double f2 = f * f;
  if (model == ORA_IDIV) {
    double a = 1.0 + tau * lam1;
    double s = sqrt(xh * xh + 4.0 * a * tau * lam1 * f2);
    *out = (xh >= 0.0) ? (xh + s) / (2.0 * a) : 2.0 * tau * lam1 * f2 / (s - xh);
    return 0;
  }
  double l2 = (model == ORA_COMBINED) ? lam2 : 0.0;
  double lf = log(f);
  double lo = xh < lf ? xh : lf, hi = xh < lf ? lf : xh;
  double w = xh;
  int it;
  for (it = 1; it <= 200; ++it) {
    double em = exp(-2.0 * w), ep = exp(2.0 * w);
    double phi = w - xh + tau * lam1 * (1.0 - f2 * em) + tau * l2 * (ep - f2);
    double dphi = 1.0 + 2.0 * tau * lam1 * f2 * em + 2.0 * tau * l2 * ep;
    if (phi > 0.0) hi = w < hi ? w : hi; else lo = w > lo ? w : lo;
    double wn = w - phi / dphi;
    if (!(wn >= lo && wn <= hi)) wn = 0.5 * (lo + hi);
    double dw = wn - w;
    w = wn;
    if (fabs(dw) <= 1e-15 * (fabs(w) > 1.0 ? fabs(w) : 1.0)) break;
  }
  *out = w;
  return it;
}

int ora_prox(const double* xhat, const double* f, long n, int model, double tau, double lam1, double lam2,
             double* out, int* max_iters) {
  int mx = 0;
#pragma omp parallel for schedule(static) reduction(max : mx)
  for (long p = 0; p < n; ++p) {
    int it = prox_pixel(xhat[p], f[p], model, tau, lam1, lam2, &out[p]);
    if (it > mx) mx = it;
  }
  if (max_iters) *max_iters = mx;
  return ORA_OK;
}

static double dot_rows(const double* a, const double* b, int H, int W) {
  size_t n = (size_t)H * W;
  double* e = (double*)malloc(sizeof(double) * n);
  if (!e) return NAN;
  for (size_t p = 0; p < n; ++p) e[p] = a[p] * b[p];
  double s = sum_rows(e, H, W);
  free(e);
  return s;
}

/* One inertial forward-backward trial at step alpha:
 *   xhat = x - alpha grad + beta (x - xprev),  xnext = prox_{alpha G}(xhat). */
static void trial(const double* x, const double* xprev, const double* grad, const double* f, long n,
                  const ora_params* p, double alpha, double* xhat, double* xnext) {
  for (long q = 0; q < n; ++q) xhat[q] = x[q] - alpha * grad[q] + p->beta * (x[q] - xprev[q]);
  ora_prox(xhat, f, n, p->model, alpha, p->lam1, p->lam2, xnext, NULL);
}

/* Teacher-forced single step at a given L (no test): info = {F(x+), G(x+), s1 = <grad F(x), d>, s2 = |d|^2}. */
int ora_step(const ora_params* p, const double* f, const double* bank, const double* theta, int nf, int H, int W,
             const double* x, const double* xprev, double L, double* xnext, double* info) {
  long n = (long)H * W;
  double* g = (double*)malloc(sizeof(double) * n);
  double* xh = (double*)malloc(sizeof(double) * n);
  double* d = (double*)malloc(sizeof(double) * n);
  if (!g || !xh || !d) { free(g); free(xh); free(d); return ORA_ENOMEM; }
  ora_grad_F(x, H, W, bank, theta, nf, p->model, p->boundary, g);
  double alpha = (p->step_mode == ORA_FIXED) ? p->alpha_fixed : 1.9 * (1.0 - p->beta) / L;
  trial(x, xprev, g, f, n, p, alpha, xh, xnext);
  for (long q = 0; q < n; ++q) d[q] = xnext[q] - x[q];
  if (info) {
    info[0] = ora_energy_F(xnext, H, W, bank, theta, nf, p->model, p->boundary);
    info[1] = ora_energy_G(xnext, f, H, W, p->model, p->lam1, p->lam2);
    info[2] = dot_rows(g, d, H, W);
    info[3] = dot_rows(d, d, H, W);
  }
  free(g); free(xh); free(d);
  return ORA_OK;
}

/* iPiano with backtracking (or a fixed step), resumable: the state is
 * (x_cur = x^n, x_prev = x^{n-1}, L) and is updated in place.
 * Each iteration: L <- eta_down L; then trials alpha = 1.9 (1 - beta) / L until
 * F(x+) <= F(x) + <grad F(x), d> + L/2 |d|^2, doubling-style L <- eta_up L on a
 * rejection.  stats (nullable) receives per iteration:
 *   {F(x+), G(x+), L, alpha, trials, <grad F(x), d>, |d|^2, |x - x_prev|^2}. */
int ora_ipiano(const ora_params* p, const double* f, const double* bank, const double* theta, int nf, int H, int W,
               double* x_cur, double* x_prev, double* L_inout, int iters, double* stats) {
  long n = (long)H * W;
  double* g = (double*)malloc(sizeof(double) * n);
  double* xh = (double*)malloc(sizeof(double) * n);
  double* xn = (double*)malloc(sizeof(double) * n);
  double* d = (double*)malloc(sizeof(double) * n);
  double* m = (double*)malloc(sizeof(double) * n);
  if (!g || !xh || !xn || !d || !m) { free(g); free(xh); free(xn); free(d); free(m); return ORA_ENOMEM; }
  int status = ORA_OK;
  double L = *L_inout;
  double Fx = ora_energy_F(x_cur, H, W, bank, theta, nf, p->model, p->boundary);
  for (int it = 0; it < iters; ++it) {
    ora_grad_F(x_cur, H, W, bank, theta, nf, p->model, p->boundary, g);
    for (long q = 0; q < n; ++q) m[q] = x_cur[q] - x_prev[q];
    double mm = dot_rows(m, m, H, W);
    double alpha, Fn, s1, s2;
    int trials = 0, accepted = 0;
    if (p->step_mode == ORA_FIXED) {
      alpha = p->alpha_fixed;
      trial(x_cur, x_prev, g, f, n, p, alpha, xh, xn);
      for (long q = 0; q < n; ++q) d[q] = xn[q] - x_cur[q];
      Fn = ora_energy_F(xn, H, W, bank, theta, nf, p->model, p->boundary);
      double Gn = ora_energy_G(xn, f, H, W, p->model, p->lam1, p->lam2);
      s1 = dot_rows(g, d, H, W);
      s2 = dot_rows(d, d, H, W);
      trials = 1;
      if (!isfinite(Fn) || !isfinite(Gn) || !isfinite(s1) || !isfinite(s2)) { status = ORA_ENONFINITE; break; }
      accepted = 1;
    } else {
      L *= p->eta_down;
      for (;;) {
        alpha = 1.9 * (1.0 - p->beta) / L;
        trial(x_cur, x_prev, g, f, n, p, alpha, xh, xn);
        for (long q = 0; q < n; ++q) d[q] = xn[q] - x_cur[q];
        Fn = ora_energy_F(xn, H, W, bank, theta, nf, p->model, p->boundary);
        double Gn = ora_energy_G(xn, f, H, W, p->model, p->lam1, p->lam2);
        s1 = dot_rows(g, d, H, W);
        s2 = dot_rows(d, d, H, W);
        ++trials;
        /* a non-finite trial energy fails the descent test: rejected like any other trial */
        int finite = isfinite(Fn) && isfinite(Gn) && isfinite(s1) && isfinite(s2);
        if (finite && Fn <= Fx + s1 + 0.5 * L * s2) { accepted = 1; break; }
        if (trials > p->max_backtracks) { status = ORA_ELINESEARCH; break; }
        L *= p->eta_up;
      }
    }
    if (!accepted) break;
    if (!isfinite(Fn)) { status = ORA_ENONFINITE; break; }
    if (stats) {
      double* s = stats + (size_t)it * 8;
      s[0] = Fn;
      s[1] = ora_energy_G(xn, f, H, W, p->model, p->lam1, p->lam2);
      s[2] = L;
      s[3] = alpha;
      s[4] = trials;
      s[5] = s1;
      s[6] = s2;
      s[7] = mm;
    }
    memcpy(x_prev, x_cur, sizeof(double) * n);
    memcpy(x_cur, xn, sizeof(double) * n);
    Fx = Fn;
  }
  *L_inout = L;
  free(g); free(xh); free(xn); free(d); free(m);
  return status;
}
