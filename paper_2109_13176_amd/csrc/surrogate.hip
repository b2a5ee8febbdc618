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

// Copies N 16-byte items into LDS with all of a thread's global loads issued
// before its first LDS store (a loop that stores each item as it arrives
// waits out one memory latency per item): item i = load(i), then
// store(i, item).
template <int N, int NT, class Load, class Store>
__device__ __forceinline__ void stage16(Load load, Store store) {
  constexpr int IT = (N + NT - 1) / NT;
  uint4 v[IT];
#pragma unroll
  for (int k = 0; k < IT; k++) {
    const int i = (int)threadIdx.x + k * NT;
    v[k] = i < N ? load(i) : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < IT; k++) {
    const int i = (int)threadIdx.x + k * NT;
    if (i < N) store(i, v[k]);
  }
}

// Two arrays staged as by stage16, all loads of both issued before any store.
// Loads and stores are unconditional, item indexes clamped to the last item
// (load(i) must read in bounds for every i < N; lanes past the end store
// the last item again, the same bytes): a load or store under a lane
// condition lets the compiler sink the load into it, or wait for it before
// the next one.
template <int N1, int N2, int NT, class Load1, class Store1, class Load2, class Store2>
__device__ __forceinline__ void stage16x2(Load1 load1, Store1 store1, Load2 load2,
                                          Store2 store2) {
  constexpr int IT1 = (N1 + NT - 1) / NT, IT2 = (N2 + NT - 1) / NT;
  uint4 v1[IT1], v2[IT2];
#pragma unroll
  for (int k = 0; k < IT1; k++) v1[k] = load1(min((int)threadIdx.x + k * NT, N1 - 1));
#pragma unroll
  for (int k = 0; k < IT2; k++) v2[k] = load2(min((int)threadIdx.x + k * NT, N2 - 1));
  __builtin_amdgcn_sched_barrier(0);  // keep every load ahead of the stores
#pragma unroll
  for (int k = 0; k < IT1; k++) store1(min((int)threadIdx.x + k * NT, N1 - 1), v1[k]);
#pragma unroll
  for (int k = 0; k < IT2; k++) store2(min((int)threadIdx.x + k * NT, N2 - 1), v2[k]);
}

// Normalised first-layer input, one thread per pixel and 8-channel group:
// xn = bf16((float)((f - mean) / std)) in double arithmetic.  The backward
// pass reads xn as the first layer's input.
__global__ __launch_bounds__(256) void k_norm(const float* __restrict__ feat,
                                              const float* __restrict__ mean,
                                              const float* __restrict__ stdv,
                                              uint16_t* __restrict__ xn, int64_t items) {
  static_assert(kFeat == 16, "two 8-channel groups per pixel");
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= items) return;
  const int cq = (int)(i & 1);
  const float4 f0 = ((const float4*)feat)[2 * i], f1 = ((const float4*)feat)[2 * i + 1];
  const float4 m0 = ((const float4*)mean)[2 * cq], m1 = ((const float4*)mean)[2 * cq + 1];
  const float4 s0 = ((const float4*)stdv)[2 * cq], s1 = ((const float4*)stdv)[2 * cq + 1];
  const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
  const float mu[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
  const float sd[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
  uint16_t b[8];
#pragma unroll
  for (int j = 0; j < 8; j++) b[j] = to_bf16((float)(((double)fv[j] - (double)mu[j]) / (double)sd[j]));
  ((uint4*)xn)[i] = make_uint4((uint32_t)b[0] | ((uint32_t)b[1] << 16),
                               (uint32_t)b[2] | ((uint32_t)b[3] << 16),
                               (uint32_t)b[4] | ((uint32_t)b[5] << 16),
                               (uint32_t)b[6] | ((uint32_t)b[7] << 16));
}

template <int CIN, int TR>
__global__ __launch_bounds__(TR * 64) void k_conv_mfma(const uint16_t* __restrict__ xin,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       uint16_t* __restrict__ y, int H, int W) {
  constexpr int PS = CIN + kPad;  // LDS stride of a pixel and of a weight row
  constexpr int NT = TR * 64;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  __shared__ __attribute__((aligned(16))) uint16_t sw[32 * 9 * PS];
  __shared__ __attribute__((aligned(16))) float sb[32];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  constexpr int Q = CIN / 8;  // 8-channel groups per pixel
  constexpr int NX = (TR + 2) * (kTC + 2) * Q;
  // the bias goes through LDS with the tiles: read from memory in the
  // epilogue it would cost one more memory latency there.  Unconditional
  // (lanes past the eighth rewrite the last quarter, same bytes).
  const float4 bq = ((const float4*)bias)[min((int)threadIdx.x, 7)];
  // weights and input tile in one round of loads
  stage16x2<32 * 9 * Q, NX, NT>(
      [&](int i) { return *(const uint4*)(w + (i / Q) * CIN + (i % Q) * 8); },
      [&](int i, uint4 v) { *(uint4*)(sw + (i / Q) * PS + (i % Q) * 8) = v; },
      [&](int i) {
        // halo pixels outside the map read a clamped pixel; the store zeroes them
        const int pix = i / Q, cq = i - pix * Q;
        const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
        const int gr = min(max(r0 + tr - 1, 0), H - 1), gc = min(max(c0 + tc - 1, 0), W - 1);
        return *(const uint4*)(xin + ((int64_t)gr * W + gc) * CIN + cq * 8);
      },
      [&](int i, uint4 v) {
        const int pix = i / Q, tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
        const int gr = r0 + tr - 1, gc = c0 + tc - 1;
        // bitwise: a branch here would let the compiler sink the load into it
        const bool ok = (gr >= 0) & (gr < H) & (gc >= 0) & (gc < W);
        const uint32_t m = ok ? ~0u : 0u;
        *(uint4*)(sx + pix * PS + (i % Q) * 8) = make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
      });
  ((float4*)sb)[min((int)threadIdx.x, 7)] = bq;
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
  float bv[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int e = 0; e < 4; e++) bv[mt][e] = sb[mt * 16 + 4 * lk + e];
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
        const float z = acc[mt][nt][e] + bv[mt][e];
        o[e] = to_bf16(z > 0.0f ? z : 0.0f);
      }
      uint2 pk;
      pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
      pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
      *(uint2*)(y + ((int64_t)r * W + col) * 32 + co0) = pk;
    }
}

// Output layer (32 -> 2, no ReLU) on matrix cores, laid out as k_conv_mfma
// with one 16-row output tile whose rows 0 and 1 are the two channels (the
// A operands of rows 2..15 are zero); each wave keeps its nine A operands
// in registers.  Block = 8 rows x 64 pixels, one wave per row, the input
// tile with its halo staged in LDS.
__global__ __launch_bounds__(512) void k_conv_out(const uint16_t* __restrict__ x,
                                                  const uint16_t* __restrict__ w,
                                                  const float* __restrict__ bias,
                                                  float* __restrict__ out, int H, int W) {
  constexpr int TR = 8, CIN = 32, PS = CIN + kPad, Q = CIN / 8;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v8bf aw[9];
#pragma unroll
  for (int tap = 0; tap < 9; tap++) {
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (lr < 2) v = *(const uint4*)(w + (lr * 9 + tap) * CIN + 8 * lk);
    aw[tap] = __builtin_bit_cast(v8bf, v);
  }
  stage16<(TR + 2) * (kTC + 2) * Q, 512>(
      [&](int i) {
        const int pix = i / Q, cq = i - pix * Q;
        const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
        const int gr = r0 + tr - 1, gc = c0 + tc - 1;
        return (gr >= 0 && gr < H && gc >= 0 && gc < W)
                   ? *(const uint4*)(x + ((int64_t)gr * W + gc) * CIN + cq * 8)
                   : make_uint4(0u, 0u, 0u, 0u);
      },
      [&](int i, uint4 v) { *(uint4*)(sx + (i / Q) * PS + (i % Q) * 8) = v; });
  __syncthreads();
  v4f acc[4];
#pragma unroll
  for (int nt = 0; nt < 4; nt++) acc[nt] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int tap = 0; tap < 9; tap++) {
    const int dy = tap / 3, dx = tap - dy * 3;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const v8bf b = *(const v8bf*)(sx + ((wv + dy) * (kTC + 2) + nt * 16 + lr + dx) * PS + 8 * lk);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[tap], b, acc[nt], 0, 0, 0);
    }
  }
  // result lane: pixel column lr, rows (channels) 4 lk + e: the two channels
  // sit in the lanes with lk = 0
  const int r = r0 + wv;
  if (r >= H || lk != 0) return;
  const float b0 = bias[0], b1 = bias[1];
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    const int col = c0 + nt * 16 + lr;
    if (col < W) *(float2*)(out + ((int64_t)r * W + col) * 2) = make_float2(acc[nt][0] + b0, acc[nt][1] + b1);
  }
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
  // a thread's pairs i = t, t + 256, ... summed in that order; sixteen
  // 16-byte loads in flight per round (clamped in-bounds loads, masked adds)
  constexpr int U = 16;
  for (int i0 = threadIdx.x; i0 < nb; i0 += 256 * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) v[u] = ((const double2*)part)[min(i0 + 256 * u, nb - 1)];
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (i0 + 256 * u < nb) {
        a += v[u].x;
        b += v[u].y;
      }
    }
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
// Input gradient of the 32 -> 2 output layer, then through the ReLU of the
// layer below: dprev[p][ci] = (x[p][ci] > 0) * sum over taps t and co of
// W[co][t][ci] dz[p - offset(t)][co], on matrix cores as one GEMM with
// K = 2 t + co (18 of the 32 of v_mfma_f32_16x16x32_bf16 used; the rest
// zero): A[ci][k] = W[co][t][ci] (constant, built once per lane), B[k][p] =
// dz[p - offset(t)][co] gathered from the block's dz tile in LDS.  The loss
// gradient dz is a sign (-1, 0 or 1), exact in bf16, so the products are
// exact and fp32-accumulated.  Stored as the bf16 pair hi = bf16(dprev),
// lo = bf16(dprev - hi) that the matrix-core kernels of the layer below read.
// Block = 8 rows x 64 pixels, one wave per row.
__global__ __launch_bounds__(512) void k_bwd_data_out(const float* __restrict__ dz,
                                                      const uint16_t* __restrict__ w,
                                                      const uint16_t* __restrict__ x,
                                                      uint16_t* __restrict__ dph,
                                                      uint16_t* __restrict__ dpl, int H, int W) {
  constexpr int TR = 8, C = 32, XC = kTC + 2;
  constexpr int NP = (TR + 2) * XC, IP = (NP + 511) / 512;
  __shared__ float sdz[NP * 2];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  // the dz tile with its halo: clamped loads all in flight, zeros outside
  // the map applied at the store (lanes past the end rewrite the last pixel)
  float2 vd[IP];
#pragma unroll
  for (int k = 0; k < IP; k++) {
    const int i = min((int)threadIdx.x + k * 512, NP - 1);
    const int tr = i / XC, tc = i - tr * XC;
    const int gr = min(max(r0 + tr - 1, 0), H - 1), gc = min(max(c0 + tc - 1, 0), W - 1);
    vd[k] = *(const float2*)(dz + ((int64_t)gr * W + gc) * 2);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = r0 + wv;
  // the ReLU mask of the layer below for all of the lane's outputs
  uint2 xmv[kTC / 16][2];
#pragma unroll
  for (int nt = 0; nt < kTC / 16; nt++)
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
      xmv[nt][mt] = *(const uint2*)(x + ((int64_t)min(r, H - 1) * W + min(c0 + nt * 16 + (lane & 15), W - 1)) * C +
                                    mt * 16 + 4 * (lane >> 4));
  const int lr = lane & 15, kg = lane >> 4;
  // A: row ci = 16 mt + lr, k = 8 kg + j -> (t, co) = (k / 2, k % 2)
  v8bf a[2];
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int k = 8 * kg + j, tap = k >> 1, co = k & 1;
      const uint16_t wb = k < 18 ? w[(co * 9 + tap) * C + 16 * mt + lr] : (uint16_t)0;
      a[mt][j] = __builtin_bit_cast(__bf16, wb);
    }
#pragma unroll
  for (int k = 0; k < IP; k++) {
    const int i = min((int)threadIdx.x + k * 512, NP - 1);
    const int tr = i / XC, tc = i - tr * XC;
    const int gr = r0 + tr - 1, gc = c0 + tc - 1;
    const bool ok = (gr >= 0) & (gr < H) & (gc >= 0) & (gc < W);
    sdz[2 * i] = ok ? vd[k].x : 0.0f;
    sdz[2 * i + 1] = ok ? vd[k].y : 0.0f;
  }
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < kTC / 16; nt++) {
    const int pc = nt * 16 + lr;  // tile column of this lane's pixel
    v8bf b;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      const int k = 8 * kg + j, kk = k < 18 ? k : 0, tap = kk >> 1, co = kk & 1;
      // the output pixel p - offset(t) sees this pixel through tap t
      const int sr = wv + 1 - (tap / 3 - 1), sc = pc + 1 - (tap % 3 - 1);
      const float v = sdz[(sr * XC + sc) * 2 + co];
      b[j] = (__bf16)(k < 18 ? v : 0.0f);
    }
    v4f acc[2];
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
      acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, v4f{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
    const int col = c0 + pc;
    if (r >= H || col >= W) continue;
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
      const int ci0 = mt * 16 + 4 * kg;
      const int64_t o = ((int64_t)r * W + col) * C + ci0;
      const uint2 xm = xmv[nt][mt];
      const uint16_t xs[4] = {(uint16_t)(xm.x & 0xFFFFu), (uint16_t)(xm.x >> 16),
                              (uint16_t)(xm.y & 0xFFFFu), (uint16_t)(xm.y >> 16)};
      uint16_t hi[4], lo[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const float v = from_bf16(xs[e]) > 0.0f ? acc[mt][e] : 0.0f;
        hi[e] = to_bf16(v);
        lo[e] = to_bf16(v - from_bf16(hi[e]));
      }
      *(uint2*)(dph + o) = make_uint2((uint32_t)hi[0] | ((uint32_t)hi[1] << 16),
                                      (uint32_t)hi[2] | ((uint32_t)hi[3] << 16));
      *(uint2*)(dpl + o) = make_uint2((uint32_t)lo[0] | ((uint32_t)lo[1] << 16),
                                      (uint32_t)lo[2] | ((uint32_t)lo[3] << 16));
    }
  }
}

// Input gradient of a 32 -> 32 layer on matrix cores.  The transposed
// convolution is a forward convolution of dz with W'[ci][t][co] =
// W[co][8 - t][ci] (tap t reads dz at p + offset(t); offset(8 - t) =
// -offset(t)), masked by the ReLU of the layer below.  dz enters as two bf16
// parts, hi = bf16(dz) and lo = bf16(dz - hi), each through the same
// instructions into one fp32 accumulator, so the product keeps about 16 bits
// of dz beyond bf16.  Layout and operand lanes as k_conv_mfma (CIN = 32); the
// tile is staged twice (hi, then lo) through one LDS array.  wt holds the
// transposed weights W' (rows ci * 9 + t, 32 co each, written by k_pack);
// the result leaves as the bf16 pair of the layer below only.
template <int TR>
__global__ __launch_bounds__(TR * 64) void k_bwd_data_mfma(const uint16_t* __restrict__ dzh,
                                                           const uint16_t* __restrict__ dzl,
                                                           const uint16_t* __restrict__ wt,
                                                           const uint16_t* __restrict__ x,
                                                           uint16_t* __restrict__ dph,
                                                           uint16_t* __restrict__ dpl, int H,
                                                           int W) {
  constexpr int C = 32, PS = C + kPad, NT = TR * 64, Q = C / 8;
  constexpr int NX = (TR + 2) * (kTC + 2) * Q, IX = (NX + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) uint16_t sx[(TR + 2) * (kTC + 2) * PS];
  __shared__ __attribute__((aligned(16))) uint16_t sw[32 * 9 * PS];
  const int r0 = blockIdx.y * TR, c0 = blockIdx.x * kTC;
  // tile item i of a dz part: clamped (in-bounds) load, zero outside the map
  // applied at the store (no lane conditions around the loads)
  auto tile_load = [&](const uint16_t* src, int i) {
    const int pix = i / Q, cq = i - pix * Q;
    const int tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
    const int gr = min(max(r0 + tr - 1, 0), H - 1), gc = min(max(c0 + tc - 1, 0), W - 1);
    return *(const uint4*)(src + ((int64_t)gr * W + gc) * C + cq * 8);
  };
  auto tile_store = [&](int i, uint4 v) {
    const int pix = i / Q, tr = pix / (kTC + 2), tc = pix - tr * (kTC + 2);
    const int gr = r0 + tr - 1, gc = c0 + tc - 1;
    const uint32_t m = ((gr >= 0) & (gr < H) & (gc >= 0) & (gc < W)) ? ~0u : 0u;
    *(uint4*)(sx + pix * PS + (i % Q) * 8) = make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
  };
  // the transposed weights and the high part of dz in one round of loads
  stage16x2<32 * 9 * Q, NX, NT>(
      [&](int i) { return *(const uint4*)(wt + (i / Q) * C + (i % Q) * 8); },
      [&](int i, uint4 v) { *(uint4*)(sw + (i / Q) * PS + (i % Q) * 8) = v; },
      [&](int i) { return tile_load(dzh, i); }, tile_store);
  // the low part's loads stay in flight during the high part's products
  uint4 lo[IX];
#pragma unroll
  for (int k = 0; k < IX; k++) lo[k] = tile_load(dzl, min((int)threadIdx.x + k * NT, NX - 1));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  v4f acc[2][4];
  for (int m = 0; m < 2; m++)
    for (int n = 0; n < 4; n++) acc[m][n] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  for (int part = 0; part < 2; part++) {
    if (part == 1) {
      // (the scheduler would hoist the low part's masking into the high
      // part's products, and with it the wait for its loads)
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();  // every wave is done with the high part's tile
#pragma unroll
      for (int k = 0; k < IX; k++) tile_store(min((int)threadIdx.x + k * NT, NX - 1), lo[k]);
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
  }
  // the ReLU mask of the layer below: all eight of a lane's reads in flight
  // (clamped into the map; pixels outside it are not written)
  const int r = r0 + wv;
  uint2 xmv[2][4];
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const int col = min(c0 + nt * 16 + lr, W - 1);
      xmv[mt][nt] = *(const uint2*)(x + ((int64_t)min(r, H - 1) * W + col) * C + mt * 16 + 4 * lk);
    }
  if (r >= H) return;
#pragma unroll
  for (int mt = 0; mt < 2; mt++)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const int col = c0 + nt * 16 + lr;
      if (col >= W) continue;
      const int ci0 = mt * 16 + 4 * lk;
      const int64_t o = ((int64_t)r * W + col) * C + ci0;
      const uint2 xm = xmv[mt][nt];
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
      *(uint2*)(dph + o) = make_uint2((uint32_t)hi[0] | ((uint32_t)hi[1] << 16),
                                      (uint32_t)hi[2] | ((uint32_t)hi[3] << 16));
      *(uint2*)(dpl + o) = make_uint2((uint32_t)lo[0] | ((uint32_t)lo[1] << 16),
                                      (uint32_t)lo[2] | ((uint32_t)lo[3] << 16));
    }
}

// Weight and bias gradient partials on matrix cores: dW[co][ci][t] =
// sum_p dz[p][co] x[p + offset(t)][ci] is one GEMM per tap with A = dz^T
// (row = output channel), B = the shifted x (column = input channel) and
// K = pixels.  Both tiles stay in LDS in their memory layout (pixel rows,
// channels contiguous, stored with 16-byte loads and 8-byte LDS writes); the
// K-major operand fragments come from the LDS transpose read
// (ds_read_b64_tr_b16): within each 16-lane group, output lane s receives
// element s % 4 of the 8-byte rows read by lanes s / 4, 4 + s / 4,
// 8 + s / 4 and 12 + s / 4.  So when lane s of group g points at pixel
// p0 + 8 g + s / 4 (and + 4 for the second half), channel c0 + 4 (s % 4),
// lane s holds the 8 consecutive pixels of channel c0 + s that the 16x16x32
// operand layout asks for (A row / B column = lane % 16, k = 8 (lane / 16)
// + e).  The tap shift is a whole-pixel offset in the staged x tile.
//
// Block = 4 waves over NTILE tiles of 4 rows x 64 pixels (accumulators stay
// in registers across the tiles); wave w takes output tile pair (co tile
// w % 2, ci tile (w / 2) % (CIN / 16)) for all 9 taps and, for CIN = 16, the
// rows of parity w / 2 (the two waves of a pair are added in LDS in fixed
// order).  dz enters as the bf16 pair hi + lo of the input-gradient kernel
// of the layer above (two MFMAs per product).  The bias gradient is the same
// product with an all-ones B.  One partial [co][ci][tap] + [co] per block.
constexpr int kWgRows = 4;            // rows per tile
constexpr int kWgTiles = 4;           // tiles per block
constexpr int kWgPZ = 32 + 4;         // LDS pixel stride (bf16) of the dz tiles
typedef short v8s __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v8bf tr_pair(const uint16_t* lo4, const uint16_t* hi4) {
  const v4s a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4s*)lo4);
  const v4s b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) v4s*)hi4);
  const v8s c = __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(v8bf, c);
}

template <int CIN, int NTILE>
__global__ __launch_bounds__(256) void k_bwd_weight_mfma(const uint16_t* __restrict__ dzh,
                                                         const uint16_t* __restrict__ dzl,
                                                         const uint16_t* __restrict__ x,
                                                         float* __restrict__ part, int H, int W) {
  constexpr int CO = 32, NW = CO * CIN * 9, NCT = CIN / 16;
  constexpr int NPAIR = 2 * NCT, RSPLIT = 4 / NPAIR;  // waves per (co, ci) tile pair
  constexpr int PX = CIN + 4;                          // LDS pixel stride of the x tile
  constexpr int XC = kTC + 2, XR = kWgRows + 2;       // x tile with its halo
  static_assert(NPAIR * RSPLIT == 4, "four waves");
  __shared__ __attribute__((aligned(16))) uint16_t sdz[2 * kWgRows * kTC * kWgPZ];
  __shared__ __attribute__((aligned(16))) uint16_t sx[XR * XC * PX];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = lane & 15, g = lane >> 4;
  const int pair = wv % NPAIR, rs = wv / NPAIR;
  const int mt = pair & 1, nt = pair >> 1;
  const int c0 = blockIdx.x * kTC;
  v4f acc[9], accb = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < 9; t++) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  v8bf ones;
#pragma unroll
  for (int e = 0; e < 8; e++) ones[e] = (__bf16)1.0f;
  // Tile t's loads (both dz parts and the x tile with its halo) are issued
  // before tile t - 1's products and stored to LDS after them: clamped
  // in-bounds loads, zeros outside the map applied at the store.
  constexpr int NZ = 2 * kWgRows * kTC * 4, NXI = XR * XC * (CIN / 8);
  constexpr int IZ = (NZ + 255) / 256, IXI = (NXI + 255) / 256;
  uint4 vz[IZ], vx[IXI];
  auto load_tile = [&](int tile) {
    const int r0 = (blockIdx.y * NTILE + tile) * kWgRows;
#pragma unroll
    for (int k = 0; k < IZ; k++) {
      const int i = min((int)threadIdx.x + k * 256, NZ - 1);
      const int hl = i / (kWgRows * kTC * 4), rem = i - hl * (kWgRows * kTC * 4);
      const int pix = rem >> 2, cg = rem & 3;
      const int gr = min(r0 + pix / kTC, H - 1), gc = min(c0 + pix % kTC, W - 1);
      vz[k] = *(const uint4*)((hl ? dzl : dzh) + ((int64_t)gr * W + gc) * CO + cg * 8);
    }
#pragma unroll
    for (int k = 0; k < IXI; k++) {
      const int i = min((int)threadIdx.x + k * 256, NXI - 1);
      const int pix = i / (CIN / 8), cq = i - pix * (CIN / 8);
      const int tr = pix / XC, tc = pix - tr * XC;
      const int gr = min(max(r0 + tr - 1, 0), H - 1), gc = min(max(c0 + tc - 1, 0), W - 1);
      vx[k] = *(const uint4*)(x + ((int64_t)gr * W + gc) * CIN + cq * 8);
    }
  };
  auto store_tile = [&](int tile) {
    const int r0 = (blockIdx.y * NTILE + tile) * kWgRows;
#pragma unroll
    for (int k = 0; k < IZ; k++) {
      const int i = min((int)threadIdx.x + k * 256, NZ - 1);
      const int rem = i % (kWgRows * kTC * 4), pix = rem >> 2;
      const int gr = r0 + pix / kTC, gc = c0 + pix % kTC;
      const uint32_t m = ((gr < H) & (gc < W)) ? ~0u : 0u;
      uint2* d = (uint2*)(sdz + (i >> 2) * kWgPZ + (i & 3) * 8);
      d[0] = make_uint2(vz[k].x & m, vz[k].y & m);
      d[1] = make_uint2(vz[k].z & m, vz[k].w & m);
    }
#pragma unroll
    for (int k = 0; k < IXI; k++) {
      const int i = min((int)threadIdx.x + k * 256, NXI - 1);
      const int pix = i / (CIN / 8), tr = pix / XC, tc = pix - tr * XC;
      const int gr = r0 + tr - 1, gc = c0 + tc - 1;
      const uint32_t m = ((gr >= 0) & (gr < H) & (gc >= 0) & (gc < W)) ? ~0u : 0u;
      uint2* d = (uint2*)(sx + pix * PX + (i % (CIN / 8)) * 8);
      d[0] = make_uint2(vx[k].x & m, vx[k].y & m);
      d[1] = make_uint2(vx[k].z & m, vx[k].w & m);
    }
  };
  load_tile(0);
  for (int tile = 0; tile < NTILE; tile++) {
    // (keeps the masking of the stores below out of the previous products)
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();  // the previous tile has been read
    store_tile(tile);
    __syncthreads();
    if (tile + 1 < NTILE) load_tile(tile + 1);
    for (int r = rs; r < kWgRows; r += RSPLIT) {
#pragma unroll
      for (int kc = 0; kc < kTC / 32; kc++) {
        const int pa = r * kTC + kc * 32 + 8 * g + (s >> 2);
        const int ca = mt * 16 + 4 * (s & 3);
        const uint16_t* ah = sdz + pa * kWgPZ + ca;
        const uint16_t* al = ah + kWgRows * kTC * kWgPZ;
        const v8bf a_hi = tr_pair(ah, ah + 4 * kWgPZ);
        const v8bf a_lo = tr_pair(al, al + 4 * kWgPZ);
        if (nt == 0) {
          accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, ones, accb, 0, 0, 0);
          accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, ones, accb, 0, 0, 0);
        }
        const int cb = nt * 16 + 4 * (s & 3);
#pragma unroll
        for (int t = 0; t < 9; t++) {
          const int dy = t / 3, dx = t - dy * 3;
          const uint16_t* bp = sx + ((r + dy) * XC + kc * 32 + 8 * g + (s >> 2) + dx) * PX + cb;
          const v8bf b = tr_pair(bp, bp + 4 * PX);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_hi, b, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_lo, b, acc[t], 0, 0, 0);
        }
      }
    }
  }
  float* out = part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (NW + CO);
  if constexpr (RSPLIT == 2) {
    // the odd-row waves hand their sums to the even-row waves of the same pair
    __syncthreads();
    float* red = (float*)sdz;  // [pair][t][e][lane] + bias
    if (rs == 1) {
#pragma unroll
      for (int t = 0; t < 9; t++)
#pragma unroll
        for (int e = 0; e < 4; e++) red[((pair * 10 + t) * 4 + e) * 64 + lane] = acc[t][e];
#pragma unroll
      for (int e = 0; e < 4; e++) red[((pair * 10 + 9) * 4 + e) * 64 + lane] = accb[e];
    }
    __syncthreads();
    if (rs == 1) return;
#pragma unroll
    for (int t = 0; t < 9; t++)
#pragma unroll
      for (int e = 0; e < 4; e++) acc[t][e] += red[((pair * 10 + t) * 4 + e) * 64 + lane];
#pragma unroll
    for (int e = 0; e < 4; e++) accb[e] += red[((pair * 10 + 9) * 4 + e) * 64 + lane];
  }
  // result lane: column ci = s of the tile, rows co = 4 g + e
#pragma unroll
  for (int t = 0; t < 9; t++)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int co = mt * 16 + 4 * g + e, ci = nt * 16 + s;
      out[(co * CIN + ci) * 9 + t] = acc[t][e];
    }
  if (nt == 0 && s == 0) {
#pragma unroll
    for (int e = 0; e < 4; e++) out[NW + mt * 16 + 4 * g + e] = accb[e];
  }
}

// Weight (and bias) gradient of the 32 -> 2 output layer on matrix cores,
// laid out as k_bwd_weight_mfma: A = dz^T with the two output channels as
// rows 0 and 1 of a 16-row operand (rows 2..15 zero), staged as 16-channel
// pixel rows; dz is the loss gradient, a sign (-1, 0 or 1) exact in bf16, so
// one product per pair.  Wave w takes ci tile w % 2 and the rows of parity
// w / 2 (the two waves of a tile are added in LDS in fixed order).
template <int NTILE>
__global__ __launch_bounds__(256) void k_bwd_weight_out(const float* __restrict__ dz,
                                                        const uint16_t* __restrict__ x,
                                                        float* __restrict__ part, int H, int W) {
  constexpr int CIN = 32, CO = 2, NW = CO * CIN * 9, PZ = 16 + 4, PX = CIN + 4;
  constexpr int XC = kTC + 2, XR = kWgRows + 2;
  __shared__ __attribute__((aligned(16))) uint16_t sdz[kWgRows * kTC * PZ];
  __shared__ __attribute__((aligned(16))) uint16_t sx[XR * XC * PX];
  __shared__ float red[2][10][4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = lane & 15, g = lane >> 4;
  const int nt = wv & 1, rs = wv >> 1;
  const int c0 = blockIdx.x * kTC;
  for (int i = threadIdx.x; i < kWgRows * kTC * PZ / 2; i += 256) ((uint32_t*)sdz)[i] = 0u;
  v4f acc[9], accb = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < 9; t++) acc[t] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
  v8bf ones;
#pragma unroll
  for (int e = 0; e < 8; e++) ones[e] = (__bf16)1.0f;
  // Tile t's loads (dz, one pixel per thread, and the x tile with its halo)
  // are issued before tile t - 1's products and stored to LDS after them:
  // clamped in-bounds loads, zeros outside the map applied at the store.
  static_assert(kWgRows * kTC == 256, "one dz pixel per thread");
  constexpr int NXI = XR * XC * (CIN / 8), IXI = (NXI + 255) / 256;
  float2 vz;
  uint4 vx[IXI];
  auto load_tile = [&](int tile) {
    const int r0 = (blockIdx.y * NTILE + tile) * kWgRows;
    const int pix = threadIdx.x;
    vz = *(const float2*)(dz + ((int64_t)min(r0 + pix / kTC, H - 1) * W + min(c0 + pix % kTC, W - 1)) * CO);
#pragma unroll
    for (int k = 0; k < IXI; k++) {
      const int i = min((int)threadIdx.x + k * 256, NXI - 1);
      const int pix = i / (CIN / 8), cq = i - pix * (CIN / 8);
      const int tr = pix / XC, tc = pix - tr * XC;
      const int gr = min(max(r0 + tr - 1, 0), H - 1), gc = min(max(c0 + tc - 1, 0), W - 1);
      vx[k] = *(const uint4*)(x + ((int64_t)gr * W + gc) * CIN + cq * 8);
    }
  };
  auto store_tile = [&](int tile) {
    const int r0 = (blockIdx.y * NTILE + tile) * kWgRows;
    const int pix = threadIdx.x;
    const bool zok = (r0 + pix / kTC < H) & (c0 + pix % kTC < W);
    const float2 v = zok ? vz : make_float2(0.0f, 0.0f);
    *(uint32_t*)(sdz + pix * PZ) = (uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16);
#pragma unroll
    for (int k = 0; k < IXI; k++) {
      const int i = min((int)threadIdx.x + k * 256, NXI - 1);
      const int pix = i / (CIN / 8), tr = pix / XC, tc = pix - tr * XC;
      const int gr = r0 + tr - 1, gc = c0 + tc - 1;
      const uint32_t m = ((gr >= 0) & (gr < H) & (gc >= 0) & (gc < W)) ? ~0u : 0u;
      uint2* d = (uint2*)(sx + pix * PX + (i % (CIN / 8)) * 8);
      d[0] = make_uint2(vx[k].x & m, vx[k].y & m);
      d[1] = make_uint2(vx[k].z & m, vx[k].w & m);
    }
  };
  load_tile(0);
  for (int tile = 0; tile < NTILE; tile++) {
    // (keeps the masking of the stores below out of the previous products)
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();  // the previous tile has been read (and the zero fill is done)
    store_tile(tile);
    __syncthreads();
    if (tile + 1 < NTILE) load_tile(tile + 1);
    for (int r = rs; r < kWgRows; r += 2) {
#pragma unroll
      for (int kc = 0; kc < kTC / 32; kc++) {
        const uint16_t* ap = sdz + (r * kTC + kc * 32 + 8 * g + (s >> 2)) * PZ + 4 * (s & 3);
        const v8bf a = tr_pair(ap, ap + 4 * PZ);
        if (nt == 0) accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ones, accb, 0, 0, 0);
        const int cb = nt * 16 + 4 * (s & 3);
#pragma unroll
        for (int t = 0; t < 9; t++) {
          const int dy = t / 3, dx = t - dy * 3;
          const uint16_t* bp = sx + ((r + dy) * XC + kc * 32 + 8 * g + (s >> 2) + dx) * PX + cb;
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, tr_pair(bp, bp + 4 * PX), acc[t], 0, 0, 0);
        }
      }
    }
  }
  // the odd-row waves hand their sums to the even-row waves of the same tile
  if (rs == 1) {
#pragma unroll
    for (int t = 0; t < 9; t++)
#pragma unroll
      for (int e = 0; e < 4; e++) red[nt][t][e][lane] = acc[t][e];
#pragma unroll
    for (int e = 0; e < 4; e++) red[nt][9][e][lane] = accb[e];
  }
  __syncthreads();
  if (rs == 1 || g != 0) return;  // rows co = 4 g + e: only g = 0, e < 2 exist
  float* out = part + (int64_t)(blockIdx.y * gridDim.x + blockIdx.x) * (NW + CO);
#pragma unroll
  for (int e = 0; e < CO; e++) {
    const int ci = nt * 16 + s;
#pragma unroll
    for (int t = 0; t < 9; t++) out[(e * CIN + ci) * 9 + t] = acc[t][e] + red[nt][t][e][lane];
    if (nt == 0 && s == 0) out[NW + e] = accb[e] + red[nt][9][e][lane];
  }
}


// Fixed-order (deterministic) reduction of the weight-gradient partials of
// every layer in one launch, scaled by 1 / count: layer l's partials sit at
// part + nb * off[l], one row of the layer's lp parameters per weight-gradient
// block.  A block takes 64 parameters (one per lane, possibly of two
// layers); wave w of its kRedWaves sums the partials w, w + kRedWaves, ... in
// order in double, with eight loads in flight, and the wave sums are added in
// a fixed order.
constexpr int kRedWaves = 16;

struct RedArgs {
  const float* part;
  int nb;                  // partials per parameter (weight-gradient blocks)
  int64_t off[kNL + 1];    // first parameter of each layer; off[kNL] = all
  const double* scal;
  float* grad;
};

__global__ __launch_bounds__(kRedWaves * 64) void k_reduce_grad(const RedArgs r) {
  __shared__ double ws[kRedWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t o = (int64_t)blockIdx.x * 64 + lane;
  const int nb = r.nb;
  double s = 0.0;
  if (o < r.off[kNL]) {
    int l = 0;
#pragma unroll
    for (int k = 1; k < kNL; k++) l += o >= r.off[k];
    const int64_t lp = r.off[l + 1] - r.off[l];
    const float* base = r.part + (int64_t)nb * r.off[l] + (o - r.off[l]);
    constexpr int U = 8;
    for (int b0 = w; b0 < nb; b0 += kRedWaves * U) {
      // clamped loads (in bounds, no lane condition to wait on), masked adds
      float v[U];
#pragma unroll
      for (int u = 0; u < U; u++) v[u] = base[(int64_t)min(b0 + kRedWaves * u, nb - 1) * lp];
#pragma unroll
      for (int u = 0; u < U; u++) s += b0 + kRedWaves * u < nb ? (double)v[u] : 0.0;
    }
  }
  ws[w][lane] = s;
  __syncthreads();
  if (w == 0 && o < r.off[kNL]) {
    double t = 0.0;
    for (int k = 0; k < kRedWaves; k++) t += ws[k][lane];
    r.grad[o] = (float)(t * r.scal[1]);
  }
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
// wtr (null for layers without a matrix-core input gradient): the same
// weights transposed for it, wtr[(ci * 9 + t) * cout + co] = W[co][8 - t][ci].
// One launch packs every layer: blockIdx.y = layer.
struct PackArgs {
  const float* master[kNL];
  uint16_t* wbf[kNL];
  float* bias[kNL];
  uint16_t* wtr[kNL];
};

__global__ __launch_bounds__(256) void k_pack(PackArgs pa) {
  const int l = blockIdx.y, cin = kCin[l], cout = kCout[l];
  const float* master = pa.master[l];
  uint16_t* wbf = pa.wbf[l];
  uint16_t* wtr = pa.wtr[l];
  float* bias = pa.bias[l];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nw = cout * cin * 9;
  if (i < nw) {
    const int co = i / (cin * 9), rest = i - co * cin * 9;
    const int ci = rest / 9, tap = rest - ci * 9;
    const uint16_t b = to_bf16(master[i]);
    wbf[(co * 9 + tap) * cin + ci] = b;
    if (wtr) wtr[(ci * 9 + (8 - tap)) * cout + co] = b;
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
  uint16_t* wtr[kNL];  // transposed copies for the matrix-core input gradient (else null)
  float* bias[kNL];
  uint16_t* act[kNL];  // input of each layer (bf16)
  float* out;
  float* dz0;          // fp32 loss gradient image (2 channels)
  uint16_t *dzh[2], *dzl[2];  // the same as bf16 pairs hi + lo (32 channels)
  float* part;         // weight-gradient partials, one per 16 x 16 tile
  int part_blocks;
  double* lpart;
  double* scal;
  float* mean;
  float* stdv;
  int64_t t;           // Adam step
};

namespace {

hipError_t pack_all(sgt_net_t* n) {
  PackArgs pa;
  int most = 0;
  for (int l = 0; l < kNL; l++) {
    pa.master[l] = n->master + n->off[l];
    pa.wbf[l] = n->wbf[l];
    pa.bias[l] = n->bias[l];
    pa.wtr[l] = n->wtr[l];
    const int cnt = kCout[l] * kCin[l] * 9 + kCout[l];
    if (blocks_for(cnt) > most) most = blocks_for(cnt);
  }
  hipLaunchKernelGGL(k_pack, dim3(most, kNL), dim3(256), 0, n->stream, pa);
  return hipGetLastError();
}

int32_t st_of(hipError_t e) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return MAP_E_DEVICE;
  }
  return MAP_OK;
}

// Forward of all layers; the output layer writes `out` (n->out for training,
// the caller's buffer for inference).
hipError_t forward_all(sgt_net_t* n, const float* feat, float* out) {
  const int H = n->H, W = n->W;
  dim3 g4((W + kTC - 1) / kTC, (H + 3) / 4), g8((W + kTC - 1) / kTC, (H + 7) / 8);
  const int64_t items = (int64_t)H * W * 2;
  hipLaunchKernelGGL(k_norm, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, n->stream, feat,
                     n->mean, n->stdv, n->act[0], items);
  hipLaunchKernelGGL((k_conv_mfma<16, 4>), g4, dim3(256), 0, n->stream, n->act[0], n->wbf[0],
                     n->bias[0], n->act[1], H, W);
  for (int l = 1; l < 4; l++)
    hipLaunchKernelGGL((k_conv_mfma<32, 8>), g8, dim3(512), 0, n->stream, n->act[l], n->wbf[l],
                       n->bias[l], n->act[l + 1], H, W);
  hipLaunchKernelGGL(k_conv_out, g8, dim3(512), 0, n->stream, n->act[4], n->wbf[4], n->bias[4],
                     out, H, W);
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
  // partial slots: one per block of the weight-gradient kernels
  n->part_blocks = ((W + kTC - 1) / kTC) * ((H + kWgRows * kWgTiles - 1) / (kWgRows * kWgTiles));
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
    if (l >= 1 && l <= 3) al((void**)&n->wtr[l], (size_t)kCout[l] * kCin[l] * 9 * 2);
    al((void**)&n->bias[l], (size_t)kCout[l] * 4);
    al((void**)&n->act[l], (size_t)P * kCin[l] * 2);
  }
  al((void**)&n->out, P * 2 * 4);
  al((void**)&n->dz0, P * 2 * 4);
  for (int k = 0; k < 2; k++) {
    al((void**)&n->dzh[k], P * 32 * 2);
    al((void**)&n->dzl[k], P * 32 * 2);
  }
  al((void**)&n->part, (size_t)n->part_blocks * n->np * 4);  // every layer's partials
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
  void* ps[] = {n->master, n->m, n->v, n->grad, n->out, n->dz0, n->part,
                n->lpart, n->scal, n->mean, n->stdv};
  for (void* p : ps) (void)gvom::dev_free(p);
  for (int k = 0; k < 2; k++) {
    (void)gvom::dev_free(n->dzh[k]);
    (void)gvom::dev_free(n->dzl[k]);
  }
  for (int l = 0; l < kNL; l++) {
    (void)gvom::dev_free(n->wbf[l]);
    (void)gvom::dev_free(n->wtr[l]);
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
  return st_of(forward_all(n, feat_dev, out_dev));
}

int32_t sgt_loss_grad(sgt_net_t* n, const float* feat_dev, const float* label_dev,
                      float* loss_host, float* grad_host) {
  if (!n || !feat_dev || !label_dev) return MAP_E_INVALID;
  const int H = n->H, W = n->W;
  const int64_t P = (int64_t)H * W;
  hipError_t e = forward_all(n, feat_dev, n->out);
  if (e != hipSuccess) return st_of(e);
  const int lb = blocks_for(P * 2) < 4096 ? blocks_for(P * 2) : 4096;
  hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, n->stream, n->out, label_dev, P * 2, n->dz0,
                     n->lpart);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, n->stream, n->lpart, lb, n->scal);
  const float* dz = n->dz0;  // the loss gradient (the output layer's dz)
  int hb = 0;  // bf16 pair holding dz (set by the layer above)
  dim3 g8((W + kTC - 1) / kTC, (H + 7) / 8);
  for (int l = kNL - 1; l >= 0; l--) {
    // weight gradients: the 2-channel output layer on the VALU, the others on
    // matrix cores (dz of those comes as the bf16 pair of the layer above)
    int nb;
    const dim3 gw((W + kTC - 1) / kTC, (H + kWgRows * kWgTiles - 1) / (kWgRows * kWgTiles));
    nb = (int)(gw.x * gw.y);
    float* const part = n->part + (size_t)nb * n->off[l];  // this layer's partials
    if (l == 4) {
      hipLaunchKernelGGL((k_bwd_weight_out<kWgTiles>), gw, dim3(256), 0, n->stream, dz,
                         n->act[l], part, H, W);
    } else {
      if (l == 0)
        hipLaunchKernelGGL((k_bwd_weight_mfma<16, kWgTiles>), gw, dim3(256), 0, n->stream,
                           n->dzh[hb], n->dzl[hb], n->act[l], part, H, W);
      else
        hipLaunchKernelGGL((k_bwd_weight_mfma<32, kWgTiles>), gw, dim3(256), 0, n->stream,
                           n->dzh[hb], n->dzl[hb], n->act[l], part, H, W);
    }
    if (l == 0) {
      // every layer's partials in one reduction
      RedArgs ra;
      ra.part = n->part;
      ra.nb = nb;
      for (int k = 0; k < kNL; k++) ra.off[k] = n->off[k];
      ra.off[kNL] = n->np;
      ra.scal = n->scal;
      ra.grad = n->grad;
      hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((n->np + 63) / 64)), dim3(kRedWaves * 64),
                         0, n->stream, ra);
      break;
    }
    if (l == 4)
      hipLaunchKernelGGL(k_bwd_data_out, g8, dim3(512), 0, n->stream, dz, n->wbf[l], n->act[l],
                         n->dzh[hb], n->dzl[hb], H, W);
    else
      hipLaunchKernelGGL((k_bwd_data_mfma<8>), g8, dim3(512), 0, n->stream, n->dzh[hb],
                         n->dzl[hb], n->wtr[l], n->act[l], n->dzh[hb ^ 1], n->dzl[hb ^ 1],
                         H, W);
    if (l != 4) hb ^= 1;
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
