// Learned gap-fill surrogate (a project extension, not part of the paper's
// method): per-column features of a map, a 5-layer 3x3 convolution network
// (16 -> 32 -> 32 -> 32 -> 32 -> 2 channels, ReLU, zero padding) with bf16
// weights and fp32 accumulation predicting ground height and roughness, its
// training (masked L1 loss, backward passes, Adam) and the fallback merge that
// keeps the plain per-column estimate wherever the network is not trusted.
//
// Layouts: images are [H][W][C] (channel fastest), H = nx, W = ny of the map.
// Parameters (fp32 master copy) per layer: W[co][ci][ky][kx] then b[co];
// the bf16 copy used by the kernels is W[co][tap][ci] (tap = 3 ky + kx).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <random>

#include "map_state.h"

using gvom::col_base;
using gvom::Dims;

namespace {

constexpr int kNL = 5;
constexpr int kCin[kNL] = {16, 32, 32, 32, 32};
constexpr int kCout[kNL] = {32, 32, 32, 32, 2};
constexpr int kFeat = 16;
constexpr uint32_t kQNaN = 0x7FC00000u;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

int64_t layer_params(int l) { return (int64_t)kCout[l] * kCin[l] * 9 + kCout[l]; }

__host__ __device__ inline uint16_t to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int32_t wrap_add(int32_t s, int32_t n) { return s >= n ? s - n : s; }

// ---------------------------------------------------------------- features
struct FeatArgs {
  Dims d;
  const int32_t* hits;
  const int32_t* passes;
  const int32_t* minqz;
  const unsigned long long* occ;
  int32_t O[3];
  double res;
  double sx, sy, sz;  // sensor position, m
  const float* height;
  const float* density;
  const float* slope;
  const float* rough;
  const uint8_t* flags;
  const uint8_t* thin;  // may be null
  float* feat;          // [nx][ny][16]
};

// One lane per window-local column.  Features (undefined values are 0):
//  0 sum of hits, 1 sum of passes, 2 occupied voxels, 3 occupied fraction,
//  4 ground height, 5 height of the highest occupied voxel, 6 mean of the
//  occupied voxels' lowest returns, 7 height defined, 8 density of the ground
//  voxel, 9 obstacle-band density, 10 slope, 11 roughness, 12 slope defined,
//  13 horizontal distance of the column centre to the sensor, 14 sensor height
//  above the ground, 15 column thinned.  A thinned column keeps only 13, 15.
__global__ __launch_bounds__(256) void k_features(FeatArgs a) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nx * ny) return;
  const int x = c / ny, y = c - x * ny;
  float f[kFeat];
  for (int k = 0; k < kFeat; k++) f[k] = 0.0f;
  const double cx = ((double)(a.O[0] + x) + 0.5) * a.res - a.sx;
  const double cy = ((double)(a.O[1] + y) + 0.5) * a.res - a.sy;
  f[13] = (float)sqrt(cx * cx + cy * cy);
  const bool thinned = a.thin && a.thin[c];
  if (thinned) {
    f[15] = 1.0f;
  } else {
    const int sxs = wrap_add(x + a.d.ro[0], nx), sys = wrap_add(y + a.d.ro[1], ny);
    const int64_t cb = col_base(a.d, sxs, sys);
    int64_t sh = 0, sp = 0, sq = 0;
    int cnt = 0, top = -1, bottom = -1;
    for (int z = 0; z < nz; z++) {
      const int64_t e = cb + ((int64_t)wrap_add(z + a.d.ro[2], nz) << 4);
      const int32_t h = a.hits[e];
      sh += h;
      sp += a.passes[e];
      if (h >= 1) {
        cnt++;
        sq += a.minqz[e];
        if (bottom < 0) bottom = z;
        top = z;
      }
    }
    const double q2m = a.res / 65536.0;
    f[0] = (float)(double)sh;
    f[1] = (float)(double)sp;
    f[2] = (float)cnt;
    f[3] = (float)((double)cnt / (double)nz);
    const uint8_t fl = a.flags[c];
    if (fl & 1) {
      f[4] = a.height[c];
      f[7] = 1.0f;
      f[14] = (float)(a.sz - (double)a.height[c]);
    }
    if (cnt > 0) {
      const int64_t et = cb + ((int64_t)wrap_add(top + a.d.ro[2], nz) << 4);
      f[5] = (float)((double)a.minqz[et] * q2m);
      f[6] = (float)(((double)sq / (double)cnt) * q2m);
      const int64_t eb = cb + ((int64_t)wrap_add(bottom + a.d.ro[2], nz) << 4);
      const double hb = a.hits[eb], pb = a.passes[eb];
      f[8] = (float)(hb / (hb + pb));
    }
    if (fl & 2) f[9] = a.density[c];
    if (fl & 32) {
      f[10] = a.slope[c];
      f[11] = a.rough[c];
      f[12] = 1.0f;
    }
  }
  float* o = a.feat + (int64_t)c * kFeat;
  for (int k = 0; k < kFeat; k++) o[k] = f[k];
}

// Clears the voxels and occupancy of window-local columns marked in `thin`.
__global__ __launch_bounds__(256) void k_thin(Dims d, const uint8_t* thin, int32_t* hits,
                                              int32_t* passes, int32_t* minqz,
                                              unsigned long long* occ) {
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nx * ny || !thin[c]) return;
  const int x = c / ny, y = c - x * ny;
  const int sxs = wrap_add(x + d.ro[0], nx), sys = wrap_add(y + d.ro[1], ny);
  const int64_t cb = col_base(d, sxs, sys);
  for (int z = 0; z < nz; z++) {
    hits[cb + ((int64_t)z << 4)] = 0;
    passes[cb + ((int64_t)z << 4)] = 0;
    minqz[cb + ((int64_t)z << 4)] = INT32_MAX;
  }
  const int64_t col = (int64_t)sxs * ny + sys;
  occ[col * d.W] = 0;
  if (d.W > 1) occ[col * d.W + 1] = 0;
}

// Per-block sums and sums of squares of the 16 features (normalisation).
__global__ __launch_bounds__(256) void k_feat_sums(const float* feat, int64_t P, double* part) {
  __shared__ double s[2 * kFeat][256 / 64];
  double acc[2 * kFeat];
  for (int k = 0; k < 2 * kFeat; k++) acc[k] = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256)
    for (int k = 0; k < kFeat; k++) {
      const double v = feat[p * kFeat + k];
      acc[k] += v;
      acc[kFeat + k] += v * v;
    }
  for (int k = 0; k < 2 * kFeat; k++) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (__lane_id() == 0) s[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kFeat) {
    double v = 0.0;
    for (int w = 0; w < 256 / 64; w++) v += s[threadIdx.x][w];
    part[blockIdx.x * 2 * kFeat + threadIdx.x] = v;
  }
}

// ------------------------------------------------------------ forward conv
// Convolutions on matrix cores: out[co][pixel] = W[co][k] x patch[k][pixel]
// with k = (tap, ci), fp32 accumulation.  Block = TR rows x 64 pixels (one
// wave per row), input tile with a one-pixel halo and the layer's weights
// staged in LDS with a padded pixel / weight-row stride (kPad bf16), which
// spreads a wave's 8- and 16-byte reads over distinct banks.  Operand lanes:
// A row = lane % 16 (output channel), B column = lane % 16 (pixel), both
// with k = KL * (lane / 16) + e; result lane holds column lane % 16, rows
// 4 * (lane / 16) + e.
//   CIN = 16: v_mfma_f32_16x16x16_bf16 (KL = 4), one instruction per tap;
//   CIN = 32: v_mfma_f32_16x16x32_bf16 (KL = 8), one instruction per tap.
constexpr int kTC = 64, kPad = 8;

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// NORM (first layer): x holds the raw fp32 features; each is normalised as
// bf16((float)((f - mean) / std)) (double arithmetic) while staged, and the
// block's own pixels are also written to xn, the layer input the backward
// pass reads.
template <int CIN, int TR, bool NORM>
__global__ __launch_bounds__(TR * 64) void k_conv_mfma(const void* __restrict__ xin,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       uint16_t* __restrict__ y, int H, int W,
                                                       const float* __restrict__ mean,
                                                       const float* __restrict__ stdv,
                                                       uint16_t* __restrict__ xn) {
  constexpr int PS = CIN + kPad;  // LDS stride of a pixel and of a weight row
  constexpr int NT = TR * 64;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  __shared__ __attribute__((aligned(16))) uint16_t sw[32 * 9 * PS];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  constexpr int Q = CIN / 8;  // 8-channel groups per pixel
  for (int i = threadIdx.x; i < (TR + 2) * (kTC + 2) * Q; i += NT) {
    const int pix = i / Q, cq = i - pix * Q;
    const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
    const int gr = r0 + tr - 1, gc = c0 + tc - 1;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gr >= 0 && gr < H && gc >= 0 && gc < W) {
      const int64_t e = ((int64_t)gr * W + gc) * CIN + cq * 8;
      if constexpr (NORM) {
        const float* f = (const float*)xin + e;
        uint16_t b[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
          const int ch = cq * 8 + k;
          b[k] = to_bf16((float)(((double)f[k] - (double)mean[ch]) / (double)stdv[ch]));
        }
        v.x = (uint32_t)b[0] | ((uint32_t)b[1] << 16);
        v.y = (uint32_t)b[2] | ((uint32_t)b[3] << 16);
        v.z = (uint32_t)b[4] | ((uint32_t)b[5] << 16);
        v.w = (uint32_t)b[6] | ((uint32_t)b[7] << 16);
        if (tr >= 1 && tr <= TR && tc >= 1 && tc <= kTC) *(uint4*)(xn + e) = v;
      } else {
        v = *(const uint4*)((const uint16_t*)xin + e);
      }
    }
    *(uint4*)(sx + pix * PS + cq * 8) = v;
  }
  for (int i = threadIdx.x; i < 32 * 9 * Q; i += NT) {
    const int row = i / Q, cq = i - row * Q;
    *(uint4*)(sw + row * PS + cq * 8) = *(const uint4*)(w + row * CIN + cq * 8);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4f acc[2][4];
  for (int m = 0; m < 2; m++)
    for (int n = 0; n < 4; n++) acc[m][n] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int tap = 0; tap < 9; tap++) {
    const int dy = tap / 3, dx = tap - dy * 3;
    if constexpr (CIN == 32) {
      const v8bf a0 = *(const v8bf*)(sw + (lr * 9 + tap) * PS + 8 * lk);
      const v8bf a1 = *(const v8bf*)(sw + ((16 + lr) * 9 + tap) * PS + 8 * lk);
#pragma unroll
      for (int nt = 0; nt < 4; nt++) {
        const int pc = nt * 16 + lr;
        const v8bf b = *(const v8bf*)(sx + ((wv + dy) * (kTC + 2) + pc + dx) * PS + 8 * lk);
        acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][nt], 0, 0, 0);
        acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[1][nt], 0, 0, 0);
      }
    } else {
      const v4s a0 = *(const v4s*)(sw + (lr * 9 + tap) * PS + 4 * lk);
      const v4s a1 = *(const v4s*)(sw + ((16 + lr) * 9 + tap) * PS + 4 * lk);
#pragma unroll
      for (int nt = 0; nt < 4; nt++) {
        const int pc = nt * 16 + lr;
        const v4s b = *(const v4s*)(sx + ((wv + dy) * (kTC + 2) + pc + dx) * PS + 4 * lk);
        acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[0][nt], 0, 0, 0);
        acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, acc[1][nt], 0, 0, 0);
      }
    }
  }
  const int r = r0 + wv;
  if (r >= H) return;
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const int col = c0 + nt * 16 + lr;
      if (col >= W) continue;
      const int co0 = mt * 16 + 4 * lk;
      uint16_t o[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const float z = acc[mt][nt][e] + bias[co0 + e];
        o[e] = to_bf16(z > 0.0f ? z : 0.0f);
      }
      uint2 pk;
      pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
      pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
      *(uint2*)(y + ((int64_t)r * W + col) * 32 + co0) = pk;
    }
}

// Output layer (32 -> 2, no ReLU): fp32 accumulation of bf16 products, tap
// by tap and channel by channel.  Block = 8 rows x 64 pixels, one thread per
// pixel, the input tile with its halo staged in LDS.
__global__ __launch_bounds__(512) void k_conv_out(const uint16_t* __restrict__ x,
                                                  const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias,
                                                  float* __restrict__ out, int H, int W) {
  constexpr int TR = 8, PS = 32 + kPad;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  __shared__ float sw[2 * 9 * 32];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  for (int i = threadIdx.x; i < 2 * 9 * 32; i += 512) sw[i] = from_bf16(w[i]);
  for (int i = threadIdx.x; i < (TR + 2) * (kTC + 2) * 4; i += 512) {
    const int pix = i >> 2, cq = i & 3;
    const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
    const int gr = r0 + tr - 1, gc = c0 + tc - 1;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gr >= 0 && gr < H && gc >= 0 && gc < W)
      v = *(const uint4*)(x + ((int64_t)gr * W + gc) * 32 + cq * 8);
    *(uint4*)(sx + pix * PS + cq * 8) = v;
  }
  __syncthreads();
  const int tr = threadIdx.x >> 6, tc = threadIdx.x & 63;
  const int r = r0 + tr, c = c0 + tc;
  if (r >= H || c >= W) return;
  float s0 = bias[0], s1 = bias[1];
  for (int tap = 0; tap < 9; tap++) {
    const int rr = r + tap / 3 - 1, cc = c + tap % 3 - 1;
    if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
    const uint16_t* xp = sx + ((tr + tap / 3) * (kTC + 2) + tc + tap % 3) * PS;
#pragma unroll
    for (int ci = 0; ci < 32; ci++) {
      const float v = from_bf16(xp[ci]);
      s0 = __builtin_fmaf(sw[(0 * 9 + tap) * 32 + ci], v, s0);
      s1 = __builtin_fmaf(sw[(1 * 9 + tap) * 32 + ci], v, s1);
    }
  }
  out[((int64_t)r * W + c) * 2] = s0;
  out[((int64_t)r * W + c) * 2 + 1] = s1;
}


// ------------------------------------------------------------------ loss
// dz = sign(pred - label) on defined label entries (the 1/count scale is
// applied to the reduced gradients); per-block |error| sums and counts.
__global__ __launch_bounds__(256) void k_loss(const float* out, const float* label, int64_t n,
                                              float* dz, double* part) {
  double ls = 0.0, cnt = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float l = label[i];
    float g = 0.0f;
    if (!isnan(l)) {
      const float d = out[i] - l;
      ls += fabs((double)d);
      cnt += 1.0;
      g = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
    }
    dz[i] = g;
  }
  for (int o = 32; o > 0; o >>= 1) {
    ls += __shfl_xor(ls, o);
    cnt += __shfl_xor(cnt, o);
  }
  __shared__ double s[2][4];
  if (__lane_id() == 0) {
    s[0][threadIdx.x >> 6] = ls;
    s[1][threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s[0][0] + s[0][1] + s[0][2] + s[0][3];
    part[2 * blockIdx.x + 1] = s[1][0] + s[1][1] + s[1][2] + s[1][3];
  }
}

// one block: total loss and 1/count -> scal[0] = loss, scal[1] = 1/count
__global__ __launch_bounds__(256) void k_loss_total(const double* part, int nb, double* scal) {
  __shared__ double s[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s[0][threadIdx.x] = a;
  s[1][threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int i = 0; i < 256; i++) {
      ta += s[0][i];
      tb += s[1][i];
    }
    scal[0] = tb > 0.0 ? ta / tb : 0.0;
    scal[1] = tb > 0.0 ? 1.0 / tb : 0.0;
  }
}

// -------------------------------------------------------------- backward
// Input gradient of a layer, then through the ReLU of the layer below:
// dprev[p][ci] = (x[p][ci] > 0) * sum over taps, co of W[co][tap][ci] dz[p - tap][co].
// Block = 16 x 16 pixels, dz tile with halo and the weights in LDS.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_bwd_data(const float* __restrict__ dz,
                                                  const uint16_t* __restrict__ w,
                                                  const uint16_t* __restrict__ x,
                                                  float* __restrict__ dprev,
                                                  uint16_t* __restrict__ dph,
                                                  uint16_t* __restrict__ dpl, int H, int W) {
  __shared__ float sdz[18 * 18 * COUT];
  __shared__ float sw[COUT * 9 * CIN];
  const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  for (int i = threadIdx.x; i < 18 * 18 * COUT; i += 256) {
    const int pix = i / COUT, co = i - pix * COUT;
    const int gr = r0 + pix / 18 - 1, gc = c0 + pix % 18 - 1;
    sdz[i] = (gr >= 0 && gr < H && gc >= 0 && gc < W) ? dz[((int64_t)gr * W + gc) * COUT + co] : 0.0f;
  }
  for (int i = threadIdx.x; i < COUT * 9 * CIN; i += 256) sw[i] = from_bf16(w[i]);
  __syncthreads();
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int r = r0 + tr, c = c0 + tc;
  if (r >= H || c >= W) return;
  float acc[CIN];
  for (int k = 0; k < CIN; k++) acc[k] = 0.0f;
  for (int tap = 0; tap < 9; tap++) {
    // the output pixel p - (tap offset) sees this pixel through tap
    const int sr = tr + 1 - (tap / 3 - 1), sc = tc + 1 - (tap % 3 - 1);
    const float* g = sdz + (sr * 18 + sc) * COUT;
    for (int co = 0; co < COUT; co++) {
      const float gv = g[co];
      const float* wr = sw + (co * 9 + tap) * CIN;
#pragma unroll
      for (int k = 0; k < CIN; k++) acc[k] = __builtin_fmaf(wr[k], gv, acc[k]);
    }
  }
  const uint16_t* xp = x + ((int64_t)r * W + c) * CIN;
  const int64_t o = ((int64_t)r * W + c) * CIN;
  static_assert(CIN % 8 == 0, "bf16 pairs are stored 8 channels at a time");
#pragma unroll
  for (int k0 = 0; k0 < CIN; k0 += 8) {
    const uint4 xq = *(const uint4*)(xp + k0);
    const uint32_t xw[4] = {xq.x, xq.y, xq.z, xq.w};
    float v[8];
    uint32_t hw[4], lw[4];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const uint16_t xb = (uint16_t)(xw[k >> 1] >> (16 * (k & 1)));
      v[k] = from_bf16(xb) > 0.0f ? acc[k0 + k] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      // the bf16 pair the matrix-core kernels of the layer below read
      const uint16_t h0 = to_bf16(v[k]), h1 = to_bf16(v[k + 1]);
      const uint16_t l0 = to_bf16(v[k] - from_bf16(h0)), l1 = to_bf16(v[k + 1] - from_bf16(h1));
      hw[k / 2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
      lw[k / 2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    *(float4*)(dprev + o + k0) = make_float4(v[0], v[1], v[2], v[3]);
    *(float4*)(dprev + o + k0 + 4) = make_float4(v[4], v[5], v[6], v[7]);
    *(uint4*)(dph + o + k0) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    *(uint4*)(dpl + o + k0) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
  }
}

// Input gradient of a 32 -> 32 layer on matrix cores.  The transposed
// convolution is a forward convolution of dz with W'[ci][t][co] =
// W[co][8 - t][ci] (tap t reads dz at p + offset(t); offset(8 - t) =
// -offset(t)), masked by the ReLU of the layer below.  dz enters as two bf16
// parts, hi = bf16(dz) and lo = bf16(dz - hi), each through the same
// instructions into one fp32 accumulator, so the product keeps about 16 bits
// of dz beyond bf16.  Layout and operand lanes as k_conv_mfma (CIN = 32); the
// tile is staged twice (hi, then lo) through one LDS array.
template <int TR>
__global__ __launch_bounds__(TR * 64) void k_bwd_data_mfma(const uint16_t* __restrict__ dzh,
                                                           const uint16_t* __restrict__ dzl,
                                                           const uint16_t* __restrict__ w,
                                                           const uint16_t* __restrict__ x,
                                                           float* __restrict__ dprev,
                                                           uint16_t* __restrict__ dph,
                                                           uint16_t* __restrict__ dpl, int H,
                                                           int W) {
  constexpr int C = 32, PS = C + kPad, NT = TR * 64, Q = C / 8;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  __shared__ __attribute__((aligned(16))) uint16_t sw[32 * 9 * PS];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  // row ci * 9 + t of the transposed weights: W[co][8 - t][ci] over co
  for (int i = threadIdx.x; i < 32 * 9 * C; i += NT) {
    const int row = i / C, co = i - row * C;
    const int ci = row / 9, t = row - ci * 9;
    sw[row * PS + co] = w[(co * 9 + (8 - t)) * C + ci];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4f acc[2][4];
  for (int m = 0; m < 2; m++)
    for (int n = 0; n < 4; n++) acc[m][n] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int part = 0; part < 2; part++) {
    const uint16_t* src = part ? dzl : dzh;
    for (int i = threadIdx.x; i < (TR + 2) * (kTC + 2) * Q; i += NT) {
      const int pix = i / Q, cq = i - pix * Q;
      const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
      const int gr = r0 + tr - 1, gc = c0 + tc - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (gr >= 0 && gr < H && gc >= 0 && gc < W)
        v = *(const uint4*)(src + ((int64_t)gr * W + gc) * C + cq * 8);
      *(uint4*)(sx + pix * PS + cq * 8) = v;
    }
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; tap++) {
      const int dy = tap / 3, dx = tap - dy * 3;
      const v8bf a0 = *(const v8bf*)(sw + (lr * 9 + tap) * PS + 8 * lk);
      const v8bf a1 = *(const v8bf*)(sw + ((16 + lr) * 9 + tap) * PS + 8 * lk);
#pragma unroll
      for (int nt = 0; nt < 4; nt++) {
        const int pc = nt * 16 + lr;
        const v8bf b = *(const v8bf*)(sx + ((wv + dy) * (kTC + 2) + pc + dx) * PS + 8 * lk);
        acc[0][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b, acc[0][nt], 0, 0, 0);
        acc[1][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b, acc[1][nt], 0, 0, 0);
      }
    }
    __syncthreads();  // the tile is restaged for the low part
  }
  const int r = r0 + wv;
  if (r >= H) return;
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const int col = c0 + nt * 16 + lr;
      if (col >= W) continue;
      const int ci0 = mt * 16 + 4 * lk;
      const int64_t o = ((int64_t)r * W + col) * C + ci0;
      const uint2 xm = *(const uint2*)(x + o);
      const uint16_t xs[4] = {(uint16_t)(xm.x & 0xFFFFu), (uint16_t)(xm.x >> 16),
                              (uint16_t)(xm.y & 0xFFFFu), (uint16_t)(xm.y >> 16)};
      float v[4];
      uint16_t hi[4], lo[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        v[e] = from_bf16(xs[e]) > 0.0f ? acc[mt][nt][e] : 0.0f;
        hi[e] = to_bf16(v[e]);
        lo[e] = to_bf16(v[e] - from_bf16(hi[e]));
      }
      *(float4*)(dprev + o) = make_float4(v[0], v[1], v[2], v[3]);
      *(uint2*)(dph + o) = make_uint2((uint32_t)hi[0] | ((uint32_t)hi[1] << 16),
                                      (uint32_t)hi[2] | ((uint32_t)hi[3] << 16));
      *(uint2*)(dpl + o) = make_uint2((uint32_t)lo[0] | ((uint32_t)lo[1] << 16),
                                      (uint32_t)lo[2] | ((uint32_t)lo[3] << 16));
    }
}

// Weight and bias gradient partials on matrix cores, one per block of TR
// rows x 64 pixels: dW[co][ci][t] = sum_p dz[p][co] x[p + offset(t)][ci] is
// one GEMM per tap with A = dz^T (row = output channel), B = shifted x
// (column = input channel) and K = pixels.  Both are staged transposed
// (channel-major, pixels contiguous) so that a lane's 8 consecutive K values
// are one 16-byte LDS read; x is staged once per column shift dx (taps of
// equal dx share the copy).  dz enters as the bf16 pair hi + lo written by
// the input-gradient kernel of the layer above.  Wave w takes input-channel
// tile w % (CIN / 16) and every (TR * CIN / 16 / 4)-th row from w / (CIN /
// 16), so a wave keeps 9 x 2 accumulator tiles; the waves' results are
// summed in LDS in wave order (deterministic) before the partial is written.
constexpr int kWRS = kTC + 8;  // LDS row stride (bf16) of the transposed tiles

template <int CIN, int TR>
__global__ __launch_bounds__(TR * 64) void k_bwd_weight_mfma(const uint16_t* __restrict__ dzh,
                                                             const uint16_t* __restrict__ dzl,
                                                             const uint16_t* __restrict__ x,
                                                             float* __restrict__ part, int H,
                                                             int W) {
  constexpr int CO = 32, NT = TR * 64, NCT = CIN / 16;
  constexpr int NW = CO * CIN * 9;
  constexpr int NWAVE = TR, RSTEP = NWAVE / NCT;  // waves; row step of a wave
  static_assert(NWAVE % NCT == 0, "waves split evenly over the channel tiles");
  static_assert(2 * CO * TR * kWRS * 2 >= NW * 4, "the wave sum reuses the dz tile");
  __shared__ __attribute__((aligned(16))) uint16_t sdz[2 * CO * TR * kWRS];  // [hi/lo][co][row][col]
  __shared__ __attribute__((aligned(16))) uint16_t sx[CIN * (TR + 2) * kWRS];  // [ci][row][col]
  __shared__ float sbias[CO];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  for (int i = threadIdx.x; i < 2 * TR * kTC * (CO / 8); i += NT) {
    const int cg = i % (CO / 8);
    int rest = i / (CO / 8);
    const int col = rest % kTC;
    rest /= kTC;
    const int row = rest % TR, hl = rest / TR;
    const int gr = r0 + row, gc = c0 + col;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (gr < H && gc < W) v = *(const uint4*)((hl ? dzl : dzh) + ((int64_t)gr * W + gc) * CO + cg * 8);
    const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 8; k++)
      sdz[((hl * CO + cg * 8 + k) * TR + row) * kWRS + col] = (uint16_t)(q[k >> 1] >> (16 * (k & 1)));
  }
  const int nt = wv % NCT, row0 = wv / NCT;
  v4f acc[9][2];
#pragma unroll
  for (int t = 0; t < 9; t++)
#pragma unroll
    for (int m = 0; m < 2; m++) acc[t][m] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int dx = 0; dx < 3; dx++) {
    __syncthreads();  // the previous copy of x has been read
    for (int i = threadIdx.x; i < (TR + 2) * kTC * (CIN / 8); i += NT) {
      const int cg = i % (CIN / 8);
      const int rest = i / (CIN / 8);
      const int col = rest % kTC, row = rest / kTC;
      const int gr = r0 + row - 1, gc = c0 + col + dx - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (gr >= 0 && gr < H && gc >= 0 && gc < W)
        v = *(const uint4*)(x + ((int64_t)gr * W + gc) * CIN + cg * 8);
      const uint32_t q[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 8; k++)
        sx[((cg * 8 + k) * (TR + 2) + row) * kWRS + col] = (uint16_t)(q[k >> 1] >> (16 * (k & 1)));
    }
    __syncthreads();
    for (int row = row0; row < TR; row += RSTEP) {
#pragma unroll
      for (int dy = 0; dy < 3; dy++) {
        const int tap = dy * 3 + dx;
#pragma unroll
        for (int ks = 0; ks < kTC / 32; ks++) {
          const v8bf b =
              *(const v8bf*)(sx + ((nt * 16 + lr) * (TR + 2) + row + dy) * kWRS + ks * 32 + 8 * lk);
#pragma unroll
          for (int hl = 0; hl < 2; hl++)
#pragma unroll
            for (int mt = 0; mt < 2; mt++) {
              const v8bf a =
                  *(const v8bf*)(sdz + ((hl * CO + mt * 16 + lr) * TR + row) * kWRS + ks * 32 + 8 * lk);
              acc[tap][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[tap][mt], 0, 0, 0);
            }
        }
      }
    }
  }
  // bias: the block's sum of dz (hi + lo) per output channel
  if (threadIdx.x < CO) {
    float sb = 0.0f;
    for (int row = 0; row < TR; row++)
      for (int col = 0; col < kTC; col++)
        sb += from_bf16(sdz[((0 * CO + threadIdx.x) * TR + row) * kWRS + col]) +
              from_bf16(sdz[((1 * CO + threadIdx.x) * TR + row) * kWRS + col]);
    sbias[threadIdx.x] = sb;
  }
  __syncthreads();
  float* red = (float*)sdz;  // [co][ci][tap]
  for (int i = threadIdx.x; i < NW; i += NT) red[i] = 0.0f;
  __syncthreads();
  for (int w = 0; w < NWAVE; w++) {
    if (wv == w) {
#pragma unroll
      for (int t = 0; t < 9; t++)
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
          for (int e = 0; e < 4; e++) {
            const int co = mt * 16 + 4 * lk + e, ci = nt * 16 + lr;
            const int idx = (co * CIN + ci) * 9 + t;
            red[idx] += acc[t][mt][e];
          }
    }
    __syncthreads();
  }
  const int blk = blockIdx.y * gridDim.x + blockIdx.x;
  float* out = part + (int64_t)blk * (NW + CO);
  for (int i = threadIdx.x; i < NW; i += NT) out[i] = red[i];
  if (threadIdx.x < CO) out[NW + threadIdx.x] = sbias[threadIdx.x];
}

// Weight (and bias) gradient of the 32 -> 2 output layer:
// dW[co][tap][ci] = sum over pixels p of dz[p][co] x[p + off(tap)][ci].  A
// half-wave (32 lanes, lane = input channel) takes kWoCols pixels of one
// image row: it loads the 3 x (kWoCols + 2) input values of its channel
// (64 contiguous bytes across the lanes per value) and the pixels' dz at
// once, then adds up the 18 sums of its channel in column order; the block's
// eight half-waves are added in a fixed order into one partial per block
// (bias: lane 0 sums dz), so the result is reproducible.  Partial b covers
// units 8 b .. 8 b + 7 (unit = row x column chunk).
constexpr int kWoCols = 16;

__global__ __launch_bounds__(256) void k_bwd_weight_out(const float* __restrict__ dz,
                                                        const uint16_t* __restrict__ x,
                                                        float* __restrict__ part, int H, int W) {
  constexpr int CIN = 32, COUT = 2, NW = COUT * CIN * 9;
  __shared__ float red[8][NW + COUT];
  const int ci = threadIdx.x & 31, hw = threadIdx.x >> 5;
  const int chunks = (W + kWoCols - 1) / kWoCols;
  const int unit = blockIdx.x * 8 + hw;
  float acc[COUT][9];
#pragma unroll
  for (int c = 0; c < COUT; c++)
#pragma unroll
    for (int k = 0; k < 9; k++) acc[c][k] = 0.0f;
  float bsum[COUT] = {0.0f, 0.0f};
  if (unit < H * chunks) {
    const int r = unit / chunks, c0 = (unit - r * chunks) * kWoCols;
    auto ld = [&](int rr, int cc) -> float {
      return (rr >= 0 && rr < H && cc >= 0 && cc < W)
                 ? from_bf16(x[((int64_t)rr * W + cc) * CIN + ci])
                 : 0.0f;
    };
    // the chunk's 3 x (kWoCols + 2) input values and its dz, loaded up front
    // (independent loads in flight), then the sums in column order
    float xv[3][kWoCols + 2];
    float d[kWoCols][COUT];
#pragma unroll
    for (int dy = 0; dy < 3; dy++)
#pragma unroll
      for (int j = 0; j < kWoCols + 2; j++) xv[dy][j] = ld(r + dy - 1, c0 + j - 1);
#pragma unroll
    for (int j = 0; j < kWoCols; j++) {
      const bool ok = c0 + j < W;
      d[j][0] = ok ? dz[((int64_t)r * W + c0 + j) * COUT] : 0.0f;
      d[j][1] = ok ? dz[((int64_t)r * W + c0 + j) * COUT + 1] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kWoCols; j++) {
#pragma unroll
      for (int k = 0; k < 9; k++) {
        acc[0][k] = __builtin_fmaf(d[j][0], xv[k / 3][j + k % 3], acc[0][k]);
        acc[1][k] = __builtin_fmaf(d[j][1], xv[k / 3][j + k % 3], acc[1][k]);
      }
      bsum[0] += d[j][0];
      bsum[1] += d[j][1];
    }
  }
#pragma unroll
  for (int c = 0; c < COUT; c++)
#pragma unroll
    for (int k = 0; k < 9; k++) red[hw][(c * CIN + ci) * 9 + k] = acc[c][k];
  if (ci == 0) {
    red[hw][NW] = bsum[0];
    red[hw][NW + 1] = bsum[1];
  }
  __syncthreads();
  float* out = part + (int64_t)blockIdx.x * (NW + COUT);
  for (int i = threadIdx.x; i < NW + COUT; i += 256) {
    float sum = 0.0f;
    for (int g = 0; g < 8; g++) sum += red[g][i];
    out[i] = sum;
  }
}

int wo_blocks(int H, int W) { return (H * ((W + kWoCols - 1) / kWoCols) + 7) / 8; }

// Two-stage fixed-order (deterministic) reduction of the weight-gradient
// partials: stage 1 sums groups of kRedGroup consecutive tiles per parameter
// (grid.y = group), stage 2 sums the groups and scales by 1 / count.
constexpr int kRedGroup = 32;

__global__ __launch_bounds__(256) void k_reduce_parts(const float* part, int nb, int64_t np,
                                                      double* mid) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= np) return;
  const int b0 = blockIdx.y * kRedGroup, b1 = min(nb, b0 + kRedGroup);
  double s = 0.0;
  for (int b = b0; b < b1; b++) s += part[(int64_t)b * np + o];
  mid[(int64_t)blockIdx.y * np + o] = s;
}

// Stage 2: a block takes 64 parameters (one per lane); wave w sums the
// groups w, w + 4, ... in order, and the four sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_mid(const double* mid, int ng, int64_t np,
                                                    const double* scal, float* grad) {
  __shared__ double ws[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t o = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (o < np)
    for (int g = w; g < ng; g += 4) s += mid[(int64_t)g * np + o];
  ws[w][lane] = s;
  __syncthreads();
  if (w == 0 && o < np)
    grad[o] = (float)(((ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane])) * scal[1]);
}

// Adam on the fp32 master weights; the bf16 copy is repacked afterwards.
__global__ __launch_bounds__(256) void k_adam(float* w, float* m, float* v, const float* g,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// master W[co][ci][ky][kx] -> bf16 W[co][tap][ci]; biases copied (fp32)
__global__ __launch_bounds__(256) void k_pack(const float* master, int cin, int cout,
                                              uint16_t* wbf, float* bias) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nw = cout * cin * 9;
  if (i < nw) {
    const int co = i / (cin * 9), rest = i - co * cin * 9;
    const int ci = rest / 9, tap = rest - ci * 9;
    wbf[(co * 9 + tap) * cin + ci] = to_bf16(master[i]);
  } else if (i < nw + cout) {
    bias[i - nw] = master[i];
  }
}

// ---------------------------------------------------------------- fallback
// Filled height and roughness: the plain estimate where the column has one;
// elsewhere the network's, if its mean disagreement with the plain heights
// of the defined columns in the 11 x 11 window (the network's receptive
// field) is at most tol; otherwise undefined.
__global__ __launch_bounds__(256) void k_fill(const float* pred, const float* ph, const float* pr,
                                              int H, int W, double tol, float* oh, float* orr) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= (int64_t)H * W) return;
  const int r = (int)(p / W), c = (int)(p - (int64_t)r * W);
  float h = __uint_as_float(kQNaN), q = __uint_as_float(kQNaN);
  if (!isnan(ph[p])) {
    h = ph[p];
    q = pr[p];
  } else {
    double s = 0.0;
    int n = 0;
    for (int dr = -5; dr <= 5; dr++)
      for (int dc = -5; dc <= 5; dc++) {
        const int rr = r + dr, cc = c + dc;
        if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
        const int64_t k = (int64_t)rr * W + cc;
        if (isnan(ph[k])) continue;
        s += fabs((double)pred[2 * k] - (double)ph[k]);
        n++;
      }
    if (n > 0 && s / n <= tol) {
      h = pred[2 * p];
      q = fmaxf(pred[2 * p + 1], 0.0f);
    }
  }
  oh[p] = h;
  orr[p] = q;
}

int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

struct sgt_net_t {
  int H, W;
  hipStream_t stream;
  int64_t np;
  int64_t off[kNL];
  float *master, *m, *v, *grad;
  uint16_t* wbf[kNL];
  float* bias[kNL];
  uint16_t* act[kNL];  // input of each layer (bf16)
  float* out;
  float *dz0, *dz1;    // fp32 gradient images (up to 32 channels)
  uint16_t *dzh[2], *dzl[2];  // the same as bf16 pairs hi + lo (32 channels)
  float* part;         // weight-gradient partials, one per 16 x 16 tile
  double* mid;         // partials summed over groups of kRedGroup tiles
  int part_blocks;
  double* lpart;
  double* scal;
  float* mean;
  float* stdv;
  int64_t t;           // Adam step
};

namespace {

hipError_t pack_all(sgt_net_t* n) {
  for (int l = 0; l < kNL; l++) {
    const int cnt = kCout[l] * kCin[l] * 9 + kCout[l];
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(cnt)), dim3(256), 0, n->stream, n->master + n->off[l],
                       kCin[l], kCout[l], n->wbf[l], n->bias[l]);
  }
  return hipGetLastError();
}

int32_t st_of(hipError_t e) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return MAP_E_DEVICE;
  }
  return MAP_OK;
}

hipError_t forward_all(sgt_net_t* n, const float* feat) {
  const int H = n->H, W = n->W;
  dim3 g4((W + kTC - 1) / kTC, (H + 3) / 4), g8((W + kTC - 1) / kTC, (H + 7) / 8);
  hipLaunchKernelGGL((k_conv_mfma<16, 4, true>), g4, dim3(256), 0, n->stream, (const void*)feat,
                     n->wbf[0], n->bias[0], n->act[1], H, W, n->mean, n->stdv, n->act[0]);
  for (int l = 1; l < 4; l++)
    hipLaunchKernelGGL((k_conv_mfma<32, 8, false>), g8, dim3(512), 0, n->stream,
                       (const void*)n->act[l], n->wbf[l], n->bias[l], n->act[l + 1], H, W,
                       (const float*)nullptr, (const float*)nullptr, (uint16_t*)nullptr);
  hipLaunchKernelGGL(k_conv_out, g8, dim3(512), 0, n->stream, n->act[4], n->wbf[4], n->bias[4],
                     n->out, H, W);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int64_t sgt_num_params(void) {
  int64_t s = 0;
  for (int l = 0; l < kNL; l++) s += layer_params(l);
  return s;
}

int32_t sgt_destroy(sgt_net_t* n);

int32_t sgt_create(int32_t H, int32_t W, uint64_t seed, void* stream, sgt_net_t** out) {
  if (!out) return MAP_E_INVALID;
  *out = nullptr;
  if (H < 1 || W < 1 || (int64_t)H * W > (1ll << 26)) return MAP_E_INVALID;
  sgt_net_t* n = new (std::nothrow) sgt_net_t();
  if (!n) return MAP_E_OOM;
  n->H = H;
  n->W = W;
  n->stream = (hipStream_t)stream;
  n->np = sgt_num_params();
  int64_t o = 0;
  for (int l = 0; l < kNL; l++) {
    n->off[l] = o;
    o += layer_params(l);
  }
  const int64_t P = (int64_t)H * W;
  // partial slots: the larger of the 16 x 16-tile VALU kernel's count and
  // the 4-row x 64-pixel matrix-core kernel's
  n->part_blocks = ((W + 15) / 16) * ((H + 15) / 16);
  const int mfma_blocks = ((W + kTC - 1) / kTC) * ((H + 3) / 4);
  if (mfma_blocks > n->part_blocks) n->part_blocks = mfma_blocks;
  if (wo_blocks(H, W) > n->part_blocks) n->part_blocks = wo_blocks(H, W);
  int64_t maxlp = 0;
  for (int l = 0; l < kNL; l++) maxlp = layer_params(l) > maxlp ? layer_params(l) : maxlp;
  hipError_t e = hipSuccess;
  auto al = [&](void** p, size_t b) {
    if (e == hipSuccess) e = gvom::dev_alloc(p, b < 16 ? 16 : b);
  };
  al((void**)&n->master, n->np * 4);
  al((void**)&n->m, n->np * 4);
  al((void**)&n->v, n->np * 4);
  al((void**)&n->grad, n->np * 4);
  for (int l = 0; l < kNL; l++) {
    al((void**)&n->wbf[l], (size_t)kCout[l] * kCin[l] * 9 * 2);
    al((void**)&n->bias[l], (size_t)kCout[l] * 4);
    al((void**)&n->act[l], (size_t)P * kCin[l] * 2);
  }
  al((void**)&n->out, P * 2 * 4);
  al((void**)&n->dz0, P * 32 * 4);
  al((void**)&n->dz1, P * 32 * 4);
  for (int k = 0; k < 2; k++) {
    al((void**)&n->dzh[k], P * 32 * 2);
    al((void**)&n->dzl[k], P * 32 * 2);
  }
  al((void**)&n->part, (size_t)n->part_blocks * maxlp * 4);
  al((void**)&n->mid, (size_t)((n->part_blocks + kRedGroup - 1) / kRedGroup) * maxlp * 8);
  al((void**)&n->lpart, (size_t)4096 * 2 * 8);
  al((void**)&n->scal, 16);
  al((void**)&n->mean, kFeat * 4);
  al((void**)&n->stdv, kFeat * 4);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sgt_destroy(n);
    return MAP_E_OOM;
  }
  // He-normal initial weights from a seeded generator, zero biases
  std::vector<float> h(n->np, 0.0f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < kNL; l++) {
    std::normal_distribution<float> nd(0.0f, sqrtf(2.0f / (9.0f * kCin[l])));
    const int64_t nw = (int64_t)kCout[l] * kCin[l] * 9;
    for (int64_t i = 0; i < nw; i++) h[n->off[l] + i] = nd(rng);
  }
  std::vector<float> ones(kFeat, 1.0f), zeros(kFeat, 0.0f), z(n->np, 0.0f);
  e = hipMemcpy(n->master, h.data(), n->np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->m, z.data(), n->np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->v, z.data(), n->np * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->mean, zeros.data(), kFeat * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->stdv, ones.data(), kFeat * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = pack_all(n);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sgt_destroy(n);
    return MAP_E_DEVICE;
  }
  *out = n;
  return MAP_OK;
}

int32_t sgt_destroy(sgt_net_t* n) {
  if (!n) return MAP_OK;
  (void)hipStreamSynchronize(n->stream);
  void* ps[] = {n->master, n->m, n->v, n->grad, n->out, n->dz0, n->dz1, n->part, n->mid,
                n->lpart, n->scal, n->mean, n->stdv};
  for (void* p : ps) (void)gvom::dev_free(p);
  for (int k = 0; k < 2; k++) {
    (void)gvom::dev_free(n->dzh[k]);
    (void)gvom::dev_free(n->dzl[k]);
  }
  for (int l = 0; l < kNL; l++) {
    (void)gvom::dev_free(n->wbf[l]);
    (void)gvom::dev_free(n->bias[l]);
    (void)gvom::dev_free(n->act[l]);
  }
  delete n;
  return MAP_OK;
}

int32_t sgt_get_params(sgt_net_t* n, float* host) {
  if (!n || !host) return MAP_E_INVALID;
  hipError_t e = hipMemcpyAsync(host, n->master, n->np * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return st_of(e);
}

int32_t sgt_set_params(sgt_net_t* n, const float* host) {
  if (!n || !host) return MAP_E_INVALID;
  hipError_t e = hipMemcpyAsync(n->master, host, n->np * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = pack_all(n);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return st_of(e);
}

int32_t sgt_set_norm(sgt_net_t* n, const float* mean, const float* stdv) {
  if (!n || !mean || !stdv) return MAP_E_INVALID;
  for (int k = 0; k < kFeat; k++)
    if (!(stdv[k] > 0.0f) || !isfinite(mean[k]) || !isfinite(stdv[k])) return MAP_E_INVALID;
  hipError_t e = hipMemcpyAsync(n->mean, mean, kFeat * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(n->stdv, stdv, kFeat * 4, hipMemcpyHostToDevice, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  return st_of(e);
}

int32_t sgt_thin(map_t* m, const uint8_t* thin_dev) {
  if (!m || !thin_dev) return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  const int64_t C = (int64_t)m->p.nx * m->p.ny;
  m->lut_counted = false;
  m->version = gvom::next_version();
  hipLaunchKernelGGL(k_thin, dim3(blocks_for(C)), dim3(256), 0, m->stream, m->d, thin_dev, m->hits,
                     m->passes, m->minqz, m->occ);
  return st_of(hipGetLastError());
}

int32_t sgt_features(map_t* m, const map_2d_t* plain, const float sensor_xyz[3],
                     const uint8_t* thin_dev, float* feat_dev) {
  if (!m || !plain || !plain->height || !plain->slope || !plain->rough || !plain->density ||
      !plain->flags || !sensor_xyz || !feat_dev)
    return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  FeatArgs a;
  a.d = m->d;
  a.hits = m->hits;
  a.passes = m->passes;
  a.minqz = m->minqz;
  a.occ = m->occ;
  for (int i = 0; i < 3; i++) a.O[i] = m->origin[i];
  a.res = (double)m->p.res_m;
  a.sx = sensor_xyz[0];
  a.sy = sensor_xyz[1];
  a.sz = sensor_xyz[2];
  a.height = plain->height;
  a.density = plain->density;
  a.slope = plain->slope;
  a.rough = plain->rough;
  a.flags = plain->flags;
  a.thin = thin_dev;
  a.feat = feat_dev;
  const int64_t C = (int64_t)m->p.nx * m->p.ny;
  hipLaunchKernelGGL(k_features, dim3(blocks_for(C)), dim3(256), 0, m->stream, a);
  return st_of(hipGetLastError());
}

int32_t sgt_feature_sums(sgt_net_t* n, const float* feat_dev, double* sums_host) {
  if (!n || !feat_dev || !sums_host) return MAP_E_INVALID;
  const int64_t P = (int64_t)n->H * n->W;
  const int nb = 1024;
  double* part = nullptr;
  hipError_t e = gvom::dev_alloc((void**)&part, (size_t)nb * 2 * kFeat * 8);
  if (e != hipSuccess) return MAP_E_OOM;
  hipLaunchKernelGGL(k_feat_sums, dim3(nb), dim3(256), 0, n->stream, feat_dev, P, part);
  std::vector<double> h((size_t)nb * 2 * kFeat);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  (void)gvom::dev_free(part);
  if (e != hipSuccess) return st_of(e);
  for (int k = 0; k < 2 * kFeat; k++) {
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += h[(size_t)b * 2 * kFeat + k];
    sums_host[k] = s;
  }
  return MAP_OK;
}

int32_t sgt_forward(sgt_net_t* n, const float* feat_dev, float* out_dev) {
  if (!n || !feat_dev || !out_dev) return MAP_E_INVALID;
  hipError_t e = forward_all(n, feat_dev);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out_dev, n->out, (size_t)n->H * n->W * 2 * 4, hipMemcpyDeviceToDevice,
                       n->stream);
  return st_of(e);
}

int32_t sgt_loss_grad(sgt_net_t* n, const float* feat_dev, const float* label_dev,
                      float* loss_host, float* grad_host) {
  if (!n || !feat_dev || !label_dev) return MAP_E_INVALID;
  const int H = n->H, W = n->W;
  const int64_t P = (int64_t)H * W;
  hipError_t e = forward_all(n, feat_dev);
  if (e != hipSuccess) return st_of(e);
  const int lb = blocks_for(P * 2) < 4096 ? blocks_for(P * 2) : 4096;
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, n->stream, n->out, label_dev, P * 2, n->dz0,
                     n->lpart);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, n->stream, n->lpart, lb, n->scal);
  dim3 g16((W + 15) / 16, (H + 15) / 16);
  float* dz = n->dz0;
  float* dp = n->dz1;
  int hb = 0;  // bf16 pair holding dz (set by the layer above)
  dim3 g8((W + kTC - 1) / kTC, (H + 7) / 8);
  for (int l = kNL - 1; l >= 0; l--) {
    const int64_t lp = layer_params(l);
    // weight gradients: the 2-channel output layer on the VALU, the others on
    // matrix cores (dz of those comes as the bf16 pair of the layer above)
    int nb;
    if (l == 4) {
      nb = wo_blocks(H, W);
      hipLaunchKernelGGL(k_bwd_weight_out, dim3(nb), dim3(256), 0, n->stream, dz, n->act[l],
                         n->part, H, W);
    } else {
      const dim3 gw((W + kTC - 1) / kTC, (H + 3) / 4);
      if (l == 0)
        hipLaunchKernelGGL((k_bwd_weight_mfma<16, 4>), gw, dim3(256), 0, n->stream, n->dzh[hb],
                           n->dzl[hb], n->act[l], n->part, H, W);
      else
        hipLaunchKernelGGL((k_bwd_weight_mfma<32, 4>), gw, dim3(256), 0, n->stream, n->dzh[hb],
                           n->dzl[hb], n->act[l], n->part, H, W);
      nb = (int)(gw.x * gw.y);
    }
    const int ng = (nb + kRedGroup - 1) / kRedGroup;
    hipLaunchKernelGGL(k_reduce_parts, dim3(blocks_for(lp), ng), dim3(256), 0, n->stream, n->part,
                       nb, lp, n->mid);
    hipLaunchKernelGGL(k_reduce_mid, dim3((unsigned)((lp + 63) / 64)), dim3(256), 0, n->stream, n->mid, ng, lp,
                       n->scal, n->grad + n->off[l]);
    if (l == 0) break;
    if (l == 4)
      hipLaunchKernelGGL((k_bwd_data<32, 2>), g16, dim3(256), 0, n->stream, dz, n->wbf[l],
                         n->act[l], dp, n->dzh[hb], n->dzl[hb], H, W);
    else
      hipLaunchKernelGGL((k_bwd_data_mfma<8>), g8, dim3(512), 0, n->stream, n->dzh[hb],
                         n->dzl[hb], n->wbf[l], n->act[l], dp, n->dzh[hb ^ 1], n->dzl[hb ^ 1],
                         H, W);
    if (l != 4) hb ^= 1;
    float* t = dz;
    dz = dp;
    dp = t;
  }
  e = hipGetLastError();
  double scal[2] = {0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpyAsync(scal, n->scal, 16, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess && grad_host)
    e = hipMemcpyAsync(grad_host, n->grad, n->np * 4, hipMemcpyDeviceToHost, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (loss_host) *loss_host = (float)scal[0];
  return st_of(e);
}

int32_t sgt_adam(sgt_net_t* n, float lr) {
  if (!n || !(lr > 0.0f)) return MAP_E_INVALID;
  n->t++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)n->t), c2 = 1.0f - powf(b2, (float)n->t);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n->np)), dim3(256), 0, n->stream, n->master, n->m, n->v,
                     n->grad, n->np, lr, b1, b2, 1e-8f, c1, c2);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = pack_all(n);
  return st_of(e);
}

int32_t sgt_fill(const float* pred_dev, const map_2d_t* plain, int32_t H, int32_t W, float tol_m,
                 float* height_out, float* rough_out, void* stream) {
  if (!pred_dev || !plain || !plain->height || !plain->rough || !height_out || !rough_out || H < 1 ||
      W < 1 || !(tol_m >= 0.0f))
    return MAP_E_INVALID;
  const int64_t P = (int64_t)H * W;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(P)), dim3(256), 0, (hipStream_t)stream, pred_dev,
                     plain->height, plain->rough, H, W, (double)tol_m, height_out, rough_out);
  return st_of(hipGetLastError());
}

}  // extern "C"
