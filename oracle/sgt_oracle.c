/*
 * sgt_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle of the gap-fill
 * surrogate, a project extension that is not in the paper).
 *
 * Plain FP64 statement of the surrogate network and its gradient:
 *   input  x0 = features, [H][W][16] (already normalised), rounded to bf16;
 *   layers conv3x3 16->32, then 32->32 three times, then 32->2, zero padding
 *          ("same"), weights W[co][ci][3][3] rounded to bf16, biases fp32,
 *          ReLU after every layer but the last, layer inputs rounded to bf16;
 *   output [H][W][2] (ground height and roughness);
 *   loss   mean absolute error over label entries that are defined (not NaN).
 * Rounding to bf16 is round-to-nearest-even of the binary32 value; the
 * gradient treats it as the identity (straight through).  With round = 0
 * nothing is rounded, which is what the finite-difference pin checks.
 * Parameter layout: for each layer W (co, ci, ky, kx) then b (co).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NL 5
static const int CIN[NL] = {16, 32, 32, 32, 32};
static const int COUT[NL] = {32, 32, 32, 32, 2};

int64_t orc_sgt_num_params(void) {
  int64_t n = 0;
  for (int l = 0; l < NL; l++) n += (int64_t)COUT[l] * CIN[l] * 9 + COUT[l];
  return n;
}

static double bf16(double v, int round) {
  if (!round) return v;
  float f = (float)v;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return f;  /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  u &= 0xFFFF0000u;
  memcpy(&f, &u, 4);
  return f;
}

/* z[H][W][co] = sum over taps and ci of w * x[neighbour][ci] + b */
static void conv(const double* x, int H, int W, int cin, int cout, const double* w,
                 const double* b, double* z) {
  for (int i = 0; i < H; i++)
    for (int j = 0; j < W; j++)
      for (int co = 0; co < cout; co++) {
        double s = b[co];
        for (int ky = 0; ky < 3; ky++)
          for (int kx = 0; kx < 3; kx++) {
            int ii = i + ky - 1, jj = j + kx - 1;
            if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
            for (int ci = 0; ci < cin; ci++)
              s += w[((co * cin + ci) * 3 + ky) * 3 + kx] * x[((int64_t)ii * W + jj) * cin + ci];
          }
        z[((int64_t)i * W + j) * cout + co] = s;
      }
}

/* Forward pass; acts (optional) receives the input of every layer
 * (acts[l] sized H*W*CIN[l]) and pre[l] the pre-activation of every layer. */
static void forward(const float* feat, int H, int W, const float* params, int round,
                    double** acts, double** pre, double* out) {
  const int64_t P = (int64_t)H * W;
  double* x = (double*)malloc(sizeof(double) * P * 32);
  double* z = (double*)malloc(sizeof(double) * P * 32);
  for (int64_t k = 0; k < P * 16; k++) x[k] = bf16(feat[k], round);
  const float* p = params;
  for (int l = 0; l < NL; l++) {
    const int ci = CIN[l], co = COUT[l];
    double* w = (double*)malloc(sizeof(double) * co * ci * 9);
    double* b = (double*)malloc(sizeof(double) * co);
    for (int k = 0; k < co * ci * 9; k++) w[k] = bf16(p[k], round);
    p += co * ci * 9;
    for (int k = 0; k < co; k++) b[k] = p[k];
    p += co;
    if (acts) memcpy(acts[l], x, sizeof(double) * P * ci);
    conv(x, H, W, ci, co, w, b, z);
    if (pre) memcpy(pre[l], z, sizeof(double) * P * co);
    if (l < NL - 1) {
      for (int64_t k = 0; k < P * co; k++) x[k] = bf16(z[k] > 0.0 ? z[k] : 0.0, round);
    } else {
      memcpy(out, z, sizeof(double) * P * co);
    }
    free(w);
    free(b);
  }
  free(x);
  free(z);
}

int32_t orc_sgt_forward(const float* feat, int32_t H, int32_t W, const float* params,
                        int32_t round, double* out) {
  if (!feat || !params || !out || H < 1 || W < 1) return -1;
  forward(feat, H, W, params, round, NULL, NULL, out);
  return 0;
}

/* Loss (mean absolute error over defined label entries) and its gradient
 * with respect to every parameter. */
int32_t orc_sgt_loss_grad(const float* feat, int32_t H, int32_t W, const float* params,
                          const float* label, int32_t round, double* loss, double* grad) {
  if (!feat || !params || !label || !loss || !grad || H < 1 || W < 1) return -1;
  const int64_t P = (int64_t)H * W;
  double* acts[NL];
  double* pre[NL];
  for (int l = 0; l < NL; l++) {
    acts[l] = (double*)malloc(sizeof(double) * P * CIN[l]);
    pre[l] = (double*)malloc(sizeof(double) * P * COUT[l]);
  }
  double* out = (double*)malloc(sizeof(double) * P * 2);
  forward(feat, H, W, params, round, acts, pre, out);
  int64_t count = 0;
  for (int64_t k = 0; k < P * 2; k++)
    if (!isnan(label[k])) count++;
  double L = 0.0;
  double* dz = (double*)calloc((size_t)(P * 32), sizeof(double));
  for (int64_t k = 0; k < P * 2; k++) {
    if (isnan(label[k]) || count == 0) continue;
    double d = out[k] - label[k];
    L += fabs(d);
    dz[k] = (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0)) / (double)count;
  }
  *loss = count ? L / (double)count : 0.0;
  /* parameter offsets */
  int64_t off[NL];
  int64_t o = 0;
  for (int l = 0; l < NL; l++) {
    off[l] = o;
    o += (int64_t)COUT[l] * CIN[l] * 9 + COUT[l];
  }
  memset(grad, 0, sizeof(double) * o);
  double* dx = (double*)malloc(sizeof(double) * P * 32);
  for (int l = NL - 1; l >= 0; l--) {
    const int ci = CIN[l], co = COUT[l];
    const float* pw = params + off[l];
    double* gw = grad + off[l];
    double* gb = gw + (int64_t)co * ci * 9;
    /* weight and bias gradients */
    for (int i = 0; i < H; i++)
      for (int j = 0; j < W; j++)
        for (int c = 0; c < co; c++) {
          double g = dz[((int64_t)i * W + j) * co + c];
          if (g == 0.0) continue;
          gb[c] += g;
          for (int ky = 0; ky < 3; ky++)
            for (int kx = 0; kx < 3; kx++) {
              int ii = i + ky - 1, jj = j + kx - 1;
              if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
              for (int q = 0; q < ci; q++)
                gw[((c * ci + q) * 3 + ky) * 3 + kx] +=
                    g * acts[l][((int64_t)ii * W + jj) * ci + q];
            }
        }
    if (l == 0) break;
    /* input gradient, then through the ReLU of the layer below */
    for (int64_t k = 0; k < P * ci; k++) dx[k] = 0.0;
    for (int i = 0; i < H; i++)
      for (int j = 0; j < W; j++)
        for (int c = 0; c < co; c++) {
          double g = dz[((int64_t)i * W + j) * co + c];
          if (g == 0.0) continue;
          for (int ky = 0; ky < 3; ky++)
            for (int kx = 0; kx < 3; kx++) {
              int ii = i + ky - 1, jj = j + kx - 1;
              if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
              for (int q = 0; q < ci; q++)
                dx[((int64_t)ii * W + jj) * ci + q] +=
                    g * bf16(pw[((c * ci + q) * 3 + ky) * 3 + kx], round);
            }
        }
    for (int64_t k = 0; k < P * ci; k++) dz[k] = pre[l - 1][k] > 0.0 ? dx[k] : 0.0;
  }
  for (int l = 0; l < NL; l++) {
    free(acts[l]);
    free(pre[l]);
  }
  free(out);
  free(dz);
  free(dx);
  return 0;
}

/* Fallback merge.  Where the plain height is defined, the plain height and
 * roughness are kept.  Elsewhere the error estimate of the network is the
 * mean, over the plain-defined columns of the 11 x 11 window centred on the
 * column (clipped at the map edge, summed row by row in increasing order, in
 * double), of |network height - plain height|; the network's height and
 * roughness (the latter clamped at 0) are taken if that mean is <= tol_m,
 * otherwise the column stays undefined (NaN).  pred is [H][W][2]. */
int32_t orc_sgt_fill(const float* pred, const float* plain_h, const float* plain_r, int32_t H,
                     int32_t W, float tol_m, float* out_h, float* out_r) {
  if (!pred || !plain_h || !plain_r || !out_h || !out_r || H < 1 || W < 1 || !(tol_m >= 0.0f))
    return -1;
  const float nan = nanf("");
  for (int i = 0; i < H; i++)
    for (int j = 0; j < W; j++) {
      const int64_t p = (int64_t)i * W + j;
      if (!isnan(plain_h[p])) {
        out_h[p] = plain_h[p];
        out_r[p] = plain_r[p];
        continue;
      }
      double s = 0.0;
      int n = 0;
      for (int ii = i - 5; ii <= i + 5; ii++)
        for (int jj = j - 5; jj <= j + 5; jj++) {
          if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
          const int64_t k = (int64_t)ii * W + jj;
          if (isnan(plain_h[k])) continue;
          s += fabs((double)pred[2 * k] - (double)plain_h[k]);
          n++;
        }
      if (n > 0 && s / n <= (double)tol_m) {
        out_h[p] = pred[2 * p];
        out_r[p] = pred[2 * p + 1] > 0.0f ? pred[2 * p + 1] : 0.0f;
      } else {
        out_h[p] = nan;
        out_r[p] = nan;
      }
    }
  return 0;
}
