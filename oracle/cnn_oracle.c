/*
 * FP64 CPU oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.
 *
 * The network maps log f to an initial log-amplitude w0 = log f + net(log f - 4.5):
 * six 3x3 convolutions with zero "same" padding (1 -> 32, four times 32 -> 32, 32 -> 1),
 * ReLU after the first five.  The loss is the mean squared difference between w0 and the
 * target log-amplitude.  Everything here is plain nested loops in double: forward pass,
 * loss, and the gradient of the loss with respect to every weight and bias by the chain
 * rule written out layer by layer.  It shares no code with the HIP library.
 *
 * Parameter layout (the same on both sides, documented in include/foe.h): for each layer
 * l = 1..6 the weights W_l[co][ci][3][3] followed by the biases b_l[co].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CNN_LAYERS 6
static const int CNN_CIN[CNN_LAYERS] = {1, 32, 32, 32, 32, 32};
static const int CNN_COUT[CNN_LAYERS] = {32, 32, 32, 32, 32, 1};
#define CNN_SHIFT 4.5

long ora_cnn_num_params(void) {
  long n = 0;
  for (int l = 0; l < CNN_LAYERS; ++l) n += (long)CNN_COUT[l] * CNN_CIN[l] * 9 + CNN_COUT[l];
  return n;
}

/* out[co][y][x] = b[co] + sum_ci sum_{dy,dx} w[co][ci][dy][dx] in[ci][y+dy-1][x+dx-1] (zero outside). */
static void conv3(const double* in, int cin, int cout, int H, int W, const double* w, const double* b, double* out) {
  for (int co = 0; co < cout; ++co)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        double s = b[co];
        for (int ci = 0; ci < cin; ++ci)
          for (int dy = 0; dy < 3; ++dy) {
            int yy = y + dy - 1;
            if (yy < 0 || yy >= H) continue;
            for (int dx = 0; dx < 3; ++dx) {
              int xx = x + dx - 1;
              if (xx < 0 || xx >= W) continue;
              s += w[((co * cin + ci) * 3 + dy) * 3 + dx] * in[((size_t)ci * H + yy) * W + xx];
            }
          }
        out[((size_t)co * H + y) * W + x] = s;
      }
}

/* Forward pass of one image.  acts[l] (l = 0..6) receive the layer inputs/outputs:
 * acts[0] = log f - 4.5, acts[l] = relu(conv_l(acts[l-1])) for l = 1..5, acts[6] = conv_6(acts[5]).
 * Returns w0 = log f + acts[6] in w0. */
static void forward(const double* params, const double* f, int H, int W, double** acts, double* w0) {
  size_t n = (size_t)H * W;
  for (size_t p = 0; p < n; ++p) acts[0][p] = log(f[p]) - CNN_SHIFT;
  const double* prm = params;
  for (int l = 0; l < CNN_LAYERS; ++l) {
    const double* w = prm;
    const double* b = prm + CNN_COUT[l] * CNN_CIN[l] * 9;
    conv3(acts[l], CNN_CIN[l], CNN_COUT[l], H, W, w, b, acts[l + 1]);
    if (l < CNN_LAYERS - 1)
      for (size_t q = 0; q < (size_t)CNN_COUT[l] * n; ++q) acts[l + 1][q] = acts[l + 1][q] > 0.0 ? acts[l + 1][q] : 0.0;
    prm = b + CNN_COUT[l];
  }
  for (size_t p = 0; p < n; ++p) w0[p] = log(f[p]) + acts[CNN_LAYERS][p];
}

/* Loss and gradient over a batch of images (f, target amplitude u_t), each H x W:
 *   loss = (1 / (n H W)) sum (w0 - log u_t)^2.
 * grad (nullable) receives d loss / d params in the parameter layout. */
double ora_cnn_loss_grad(const double* params, const double* f, const double* ut, int nimg, int H, int W,
                         double* grad) {
  const size_t n = (size_t)H * W;
  const double scale = 1.0 / ((double)nimg * (double)n);
  double* acts[CNN_LAYERS + 1];
  for (int l = 0; l <= CNN_LAYERS; ++l) {
    int c = l == 0 ? 1 : CNN_COUT[l - 1];
    acts[l] = (double*)malloc(sizeof(double) * c * n);
  }
  double* w0 = (double*)malloc(sizeof(double) * n);
  double* d_cur = (double*)malloc(sizeof(double) * 32 * n);
  double* d_prev = (double*)malloc(sizeof(double) * 32 * n);
  long np = ora_cnn_num_params();
  if (grad) memset(grad, 0, sizeof(double) * np);
  /* offsets of each layer's parameters */
  long off[CNN_LAYERS];
  long o = 0;
  for (int l = 0; l < CNN_LAYERS; ++l) { off[l] = o; o += (long)CNN_COUT[l] * CNN_CIN[l] * 9 + CNN_COUT[l]; }
  double loss = 0.0;
  for (int im = 0; im < nimg; ++im) {
    const double* fi = f + (size_t)im * n;
    const double* ti = ut + (size_t)im * n;
    forward(params, fi, H, W, acts, w0);
    for (size_t p = 0; p < n; ++p) {
      double r = w0[p] - log(ti[p]);
      loss += r * r * scale;
      d_cur[p] = 2.0 * r * scale; /* d loss / d acts[6] */
    }
    if (!grad) continue;
    for (int l = CNN_LAYERS - 1; l >= 0; --l) {
      const int cin = CNN_CIN[l], cout = CNN_COUT[l];
      const double* w = params + off[l];
      double* gw = grad + off[l];
      double* gb = gw + cout * cin * 9;
      const double* a_in = acts[l];
      /* d_cur is d loss / d (pre-activation output of layer l) */
      for (int co = 0; co < cout; ++co)
        for (size_t p = 0; p < n; ++p) gb[co] += d_cur[(size_t)co * n + p];
      for (int co = 0; co < cout; ++co)
        for (int ci = 0; ci < cin; ++ci)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              double s = 0.0;
              for (int y = 0; y < H; ++y) {
                int yy = y + dy - 1;
                if (yy < 0 || yy >= H) continue;
                for (int x = 0; x < W; ++x) {
                  int xx = x + dx - 1;
                  if (xx < 0 || xx >= W) continue;
                  s += d_cur[((size_t)co * H + y) * W + x] * a_in[((size_t)ci * H + yy) * W + xx];
                }
              }
              gw[((co * cin + ci) * 3 + dy) * 3 + dx] += s;
            }
      if (l == 0) break;
      /* d loss / d a_in, then through the ReLU that produced a_in */
      memset(d_prev, 0, sizeof(double) * cin * n);
      for (int co = 0; co < cout; ++co)
        for (int y = 0; y < H; ++y)
          for (int x = 0; x < W; ++x) {
            double d = d_cur[((size_t)co * H + y) * W + x];
            for (int ci = 0; ci < cin; ++ci)
              for (int dy = 0; dy < 3; ++dy) {
                int yy = y + dy - 1;
                if (yy < 0 || yy >= H) continue;
                for (int dx = 0; dx < 3; ++dx) {
                  int xx = x + dx - 1;
                  if (xx < 0 || xx >= W) continue;
                  d_prev[((size_t)ci * H + yy) * W + xx] += d * w[((co * cin + ci) * 3 + dy) * 3 + dx];
                }
              }
          }
      for (size_t q = 0; q < (size_t)cin * n; ++q) d_prev[q] = a_in[q] > 0.0 ? d_prev[q] : 0.0;
      double* t = d_cur; d_cur = d_prev; d_prev = t;
    }
  }
  for (int l = 0; l <= CNN_LAYERS; ++l) free(acts[l]);
  free(w0); free(d_cur); free(d_prev);
  return loss;
}

/* Forward only: w0 of one image. */
void ora_cnn_forward(const double* params, const double* f, int H, int W, double* w0) {
  size_t n = (size_t)H * W;
  double* acts[CNN_LAYERS + 1];
  for (int l = 0; l <= CNN_LAYERS; ++l) {
    int c = l == 0 ? 1 : CNN_COUT[l - 1];
    acts[l] = (double*)malloc(sizeof(double) * c * n);
  }
  forward(params, f, H, W, acts, w0);
  for (int l = 0; l <= CNN_LAYERS; ++l) free(acts[l]);
}

/* Smallest |pre-activation| over every ReLU of the network (layers 1-5) and every pixel of the
 * batch: how close the forward pass comes to a ReLU decision that rounding could flip. */
double ora_cnn_relu_margin(const double* params, const double* f, int nimg, int H, int W) {
  size_t n = (size_t)H * W;
  double* acts[CNN_LAYERS + 1];
  for (int l = 0; l <= CNN_LAYERS; ++l) {
    int c = l == 0 ? 1 : CNN_COUT[l - 1];
    acts[l] = (double*)malloc(sizeof(double) * c * n);
  }
  double margin = INFINITY;
  for (int im = 0; im < nimg; ++im) {
    const double* fi = f + (size_t)im * n;
    for (size_t p = 0; p < n; ++p) acts[0][p] = log(fi[p]) - CNN_SHIFT;
    const double* prm = params;
    for (int l = 0; l < CNN_LAYERS - 1; ++l) {
      const double* w = prm;
      const double* b = prm + CNN_COUT[l] * CNN_CIN[l] * 9;
      conv3(acts[l], CNN_CIN[l], CNN_COUT[l], H, W, w, b, acts[l + 1]);
      for (size_t q = 0; q < (size_t)CNN_COUT[l] * n; ++q) {
        double z = acts[l + 1][q];
        if (fabs(z) < margin) margin = fabs(z);
        acts[l + 1][q] = z > 0.0 ? z : 0.0;
      }
      prm = b + CNN_COUT[l];
    }
  }
  for (int l = 0; l <= CNN_LAYERS; ++l) free(acts[l]);
  return margin;
}
