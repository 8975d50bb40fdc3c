/*
 * Driver for a sanitizer build of the FP64 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built with gcc and AddressSanitizer + UndefinedBehaviorSanitizer together with
 * foe_oracle.c and cnn_oracle.c (no OpenMP: the loops then run serially, which is
 * what the sanitizers check best).  It calls every exported oracle routine on small
 * seeded inputs, including sides below the filter radius, all three boundary
 * conditions and all three data models, so that every index path of the boundary
 * map P, the fold P^T and the line search runs at least once.  Besides the memory
 * and UB checks it asserts one property per operator that holds at any size:
 *   <K x, v> = <x, K^T v>            (the adjoint of Sec. II-C is the transpose),
 *   G(prox(xhat)) + |prox - xhat|^2 / (2 tau) <= the same at xhat (prox is a minimiser),
 *   F(x + t d) - F(x) ~ t <grad F(x), d> for small t (the gradient is F's derivative).
 * Exit status 0 when all checks pass, 1 otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t model, boundary, step_mode, max_backtracks;
  double lam1, lam2, beta, alpha_fixed, eta_up, eta_down;
} ora_params;

void ora_forward(const double* x, int H, int W, const double* k, int bc, double* y);
int ora_adjoint(const double* v, int H, int W, const double* k, int bc, double* out);
double ora_energy_F(const double* x, int H, int W, const double* bank, const double* theta, int nf, int model, int bc);
double ora_energy_G(const double* x, const double* f, int H, int W, int model, double lam1, double lam2);
int ora_grad_F(const double* x, int H, int W, const double* bank, const double* theta, int nf, int model, int bc,
               double* g);
int ora_prox(const double* xhat, const double* f, long n, int model, double tau, double lam1, double lam2, double* out,
             int* max_iters);
int ora_step(const ora_params* p, const double* f, const double* bank, const double* theta, int nf, int H, int W,
             const double* x, const double* xprev, double L, double* xnext, double* info);
int ora_ipiano(const ora_params* p, const double* f, const double* bank, const double* theta, int nf, int H, int W,
               double* x_cur, double* x_prev, double* L_inout, int iters, double* stats);
long ora_cnn_num_params(void);
double ora_cnn_loss_grad(const double* params, const double* f, const double* ut, int nimg, int H, int W,
                         double* grad);
void ora_cnn_forward(const double* params, const double* f, int H, int W, double* w0);
double ora_cnn_relu_margin(const double* params, const double* f, int nimg, int H, int W);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

/* splitmix64, mapped to [0, 1) */
static double uniform(void) {
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static double* vec(long n) {
  double* p = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

static double dot(const double* a, const double* b, long n) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static int failures = 0;

static void check(int ok, const char* what, int H, int W, int bc, int model) {
  if (!ok) {
    fprintf(stderr, "FAIL %s at %dx%d bc %d model %d\n", what, H, W, bc, model);
    failures++;
  }
}

static void run_case(int H, int W, int bc, int model, int nf) {
  const long n = (long)H * W;
  double* bank = vec(49L * nf);
  double* theta = vec(nf);
  for (long i = 0; i < 49L * nf; ++i) bank[i] = uniform() - 0.5;
  for (int i = 0; i < nf; ++i) theta[i] = 0.1 + uniform();
  double* f = vec(n);
  double* x = vec(n);
  double* v = vec(n);
  double* y = vec(n);
  double* kt = vec(n);
  for (long q = 0; q < n; ++q) {
    f[q] = 0.2 + 2.0 * uniform();
    x[q] = model == 2 ? 0.5 + uniform() : log(0.5 + uniform());
    v[q] = uniform() - 0.5;
  }

  /* forward / adjoint: transpose identity */
  ora_forward(x, H, W, bank, bc, y);
  check(ora_adjoint(v, H, W, bank, bc, kt) == 0, "adjoint status", H, W, bc, model);
  double lhs = dot(y, v, n), rhs = dot(x, kt, n);
  check(fabs(lhs - rhs) <= 1e-12 * (1.0 + fabs(lhs)), "adjoint identity", H, W, bc, model);

  /* energies and gradient: directional derivative */
  double* g = vec(n);
  double* xt = vec(n);
  check(ora_grad_F(x, H, W, bank, theta, nf, model, bc, g) == 0, "grad status", H, W, bc, model);
  double F0 = ora_energy_F(x, H, W, bank, theta, nf, model, bc);
  const double t = 1e-6;
  for (long q = 0; q < n; ++q) xt[q] = x[q] + t * v[q];
  double Fp = ora_energy_F(xt, H, W, bank, theta, nf, model, bc);
  for (long q = 0; q < n; ++q) xt[q] = x[q] - t * v[q];
  double Fm = ora_energy_F(xt, H, W, bank, theta, nf, model, bc);
  double dd = dot(g, v, n), fd = (Fp - Fm) / (2.0 * t);
  check(isfinite(F0) && fabs(fd - dd) <= 1e-5 * (1.0 + fabs(dd)), "gradient vs finite difference", H, W, bc, model);

  /* prox: the output does no worse than the input on the prox objective */
  const double lam1 = 40.0, lam2 = 0.01, tau = 0.05;
  double* xp = vec(n);
  int its = 0;
  check(ora_prox(x, f, n, model, tau, lam1, lam2, xp, &its) == 0, "prox status", H, W, bc, model);
  double Gx = ora_energy_G(x, f, H, W, model, lam1, lam2);
  double Gp = ora_energy_G(xp, f, H, W, model, lam1, lam2);
  double dist = 0.0;
  for (long q = 0; q < n; ++q) dist += (xp[q] - x[q]) * (xp[q] - x[q]);
  check(Gp + dist / (2.0 * tau) <= Gx * (1.0 + 1e-12) + 1e-12, "prox minimises", H, W, bc, model);

  /* one teacher-forced step and a few iPiano iterations (backtracking and fixed) */
  ora_params p = {model, bc, 0, 40, lam1, lam2, 0.8, 1e-3, 2.0, 1.0};
  double info[4];
  double* xn = vec(n);
  check(ora_step(&p, f, bank, theta, nf, H, W, x, x, 1.0, xn, info) == 0, "step status", H, W, bc, model);
  for (int mode = 0; mode < 2; ++mode) {
    p.step_mode = mode;
    double* xc = vec(n);
    double* xo = vec(n);
    for (long q = 0; q < n; ++q) xc[q] = xo[q] = x[q];
    double L = 1.0;
    double stats[8 * 4];
    int st = ora_ipiano(&p, f, bank, theta, nf, H, W, xc, xo, &L, 4, stats);
    check(st == 0 || st == 4, "ipiano status", H, W, bc, model);
    free(xc);
    free(xo);
  }
  free(bank); free(theta); free(f); free(x); free(v); free(y); free(kt);
  free(g); free(xt); free(xp); free(xn);
}

static void run_cnn(void) {
  const long np = ora_cnn_num_params();
  const int H = 5, W = 4, nimg = 2;
  const long n = (long)H * W;
  double* prm = vec(np);
  double* grad = vec(np);
  double* f = vec(nimg * n);
  double* ut = vec(nimg * n);
  double* w0 = vec(n);
  for (long i = 0; i < np; ++i) prm[i] = 0.2 * (uniform() - 0.5);
  for (long q = 0; q < nimg * n; ++q) {
    f[q] = 0.5 + uniform();
    ut[q] = 0.5 + uniform();
  }
  double loss = ora_cnn_loss_grad(prm, f, ut, nimg, H, W, grad);
  check(isfinite(loss) && loss >= 0.0, "cnn loss", H, W, -1, -1);
  /* directional derivative of the loss along a random parameter direction */
  double* dir = vec(np);
  double* pt = vec(np);
  for (long i = 0; i < np; ++i) dir[i] = uniform() - 0.5;
  const double t = 1e-6;
  for (long i = 0; i < np; ++i) pt[i] = prm[i] + t * dir[i];
  double lp = ora_cnn_loss_grad(pt, f, ut, nimg, H, W, NULL);
  for (long i = 0; i < np; ++i) pt[i] = prm[i] - t * dir[i];
  double lm = ora_cnn_loss_grad(pt, f, ut, nimg, H, W, NULL);
  double dd = dot(grad, dir, np), fd = (lp - lm) / (2.0 * t);
  check(fabs(fd - dd) <= 1e-5 * (1.0 + fabs(dd)), "cnn gradient vs finite difference", H, W, -1, -1);
  ora_cnn_forward(prm, f, H, W, w0);
  check(isfinite(ora_cnn_relu_margin(prm, f, nimg, H, W)), "cnn relu margin", H, W, -1, -1);
  free(prm); free(grad); free(f); free(ut); free(w0); free(dir); free(pt);
}

int main(void) {
  static const int shapes[][2] = {{1, 1}, {1, 9}, {2, 5}, {3, 3}, {4, 4}, {7, 2}, {9, 13}, {16, 5}};
  const int ns = (int)(sizeof(shapes) / sizeof(shapes[0]));
  for (int s = 0; s < ns; ++s)
    for (int bc = 0; bc < 3; ++bc)
      for (int model = 0; model < 3; ++model) run_case(shapes[s][0], shapes[s][1], bc, model, 1 + (s + bc + model) % 3);
  run_cnn();
  printf("%d cases, %d failures\n", ns * 9 + 1, failures);
  return failures ? 1 : 0;
}
