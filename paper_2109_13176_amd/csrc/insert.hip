// Scan insertion kernels: transform + return binning + exact integer ray
// traversal (Sec. III-C of arXiv 2109.13176), and the slab clears that move
// the toroidal window.
#include <math.h>

#include "gvom_internal.h"

namespace gvom {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int32_t wrap_add(int32_t s, int32_t n) { return s >= n ? s - n : s; }

// Sums an int over the 64 lanes of the wave.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One lane per point.  Each lane transforms its point, records the return in
// the end voxel, then walks the segment sensor -> point voxel by voxel and
// adds one pass to every window voxel before the end voxel.
//
// Traversal: along axis a the segment leaves its current cell when it has
// moved num_a (Q units) at speed |D_a|, i.e. at time num_a / |D_a|.  The axis
// with the smallest time steps next; times are compared exactly through the
// pairwise differences E_ab = num_a |D_b| - num_b |D_a| (int64, |.| < 2^56),
// which change only by constant increments when an axis steps.  When several
// axes share the smallest time, the axes moving up step first (the shared
// boundary belongs to the upper cell) and the axes moving down step in the
// following iteration, so the voxel at that instant is visited.
//
// Lanes of a wave step in lock-step; in each step the lanes that pass the
// same voxel as their left neighbour join its run and the run's first lane
// adds the run length with one atomic.
template <bool DISTINCT>
__global__ __launch_bounds__(kBlock) void k_insert(InsertArgs a) {
  const int lane = __lane_id();
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool in = i < a.n;
  int pidx = i;
  if (a.fw > 1 && in) {
    const int b = i / a.azimuths;
    pidx = (i - b * a.azimuths) * a.fw + b;
  }
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;

  bool nonfinite = false, outrange = false, hit = false, dhit = false, ray = false;
  int32_t q[3] = {0, 0, 0};
  if (in) {
    const float p0 = a.xyz[3 * pidx + 0];
    const float p1 = a.xyz[3 * pidx + 1];
    const float p2 = a.xyz[3 * pidx + 2];
    if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) {
      nonfinite = true;
    } else {
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = __builtin_fmaf(a.R[3 * k + 0], p0, a.t[k]);
        w = __builtin_fmaf(a.R[3 * k + 1], p1, w);
        w = __builtin_fmaf(a.R[3 * k + 2], p2, w);
        const float u = w * a.inv_r;
        const bool okk = isfinite(w) && fabsf(u) < 32768.0f;
        q[k] = okk ? (int32_t)floorf(u * 65536.0f) : 0;
        ok = ok && okk;
        const int64_t dd = (int64_t)q[k] - a.S[k];
        ok = ok && dd < (1 << 27) && -dd < (1 << 27);
      }
      if (ok) ray = true; else outrange = true;
    }
  }

  // DDA state (meaningful for ray lanes only)
  int32_t rem[3] = {0, 0, 0}, room[3] = {0, 0, 0}, sg[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
  int64_t exy = 0, exz = 0, eyz = 0;
  int64_t kxy = 0, kxz = 0, kyx = 0, kyz = 0, kzx = 0, kzy = 0;
  int32_t sidx = 0;
  if (ray) {
    const int32_t dims[3] = {nx, ny, nz};
    int32_t ad[3], num[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int32_t sv = a.S[k] >> 16;
      const int32_t ev = q[k] >> 16;
      const int32_t dq = q[k] - a.S[k];
      sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
      ad[k] = dq < 0 ? -dq : dq;
      rem[k] = ev > sv ? ev - sv : sv - ev;
      const int32_t lc = sv - a.O[k];
      room[k] = sg[k] > 0 ? dims[k] - 1 - lc : lc;
      num[k] = sg[k] > 0 ? (int32_t)((((int64_t)sv + 1) << 16) - a.S[k])
                         : (int32_t)((int64_t)a.S[k] - ((int64_t)sv << 16));
      sc[k] = wrap_add(lc + a.d.ro[k], dims[k]);
    }
    exy = (int64_t)num[0] * ad[1] - (int64_t)num[1] * ad[0];
    exz = (int64_t)num[0] * ad[2] - (int64_t)num[2] * ad[0];
    eyz = (int64_t)num[1] * ad[2] - (int64_t)num[2] * ad[1];
    kxy = (int64_t)ad[1] << 16;  // added to E_xy when x steps
    kxz = (int64_t)ad[2] << 16;
    kyx = (int64_t)ad[0] << 16;  // subtracted from E_xy when y steps
    kyz = (int64_t)ad[2] << 16;
    kzx = (int64_t)ad[0] << 16;
    kzy = (int64_t)ad[1] << 16;
    sidx = (sc[0] * ny + sc[1]) * nz + sc[2];

    // the return
    int32_t l[3];
    bool win = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      l[k] = (q[k] >> 16) - a.O[k];
      win = win && l[k] >= 0 && l[k] < dims[k];
    }
    if (win) {
      const int32_t ex = wrap_add(l[0] + a.d.ro[0], nx);
      const int32_t ey = wrap_add(l[1] + a.d.ro[1], ny);
      const int32_t ez = wrap_add(l[2] + a.d.ro[2], nz);
      const int32_t col = ex * ny + ey;
      const int32_t e = col * nz + ez;
      atomicAdd(&a.hits[e], 1);
      atomicMin(&a.minqz[e], q[2]);
      atomicOr(&a.occ[(int64_t)col * a.d.W + (ez >> 6)], 1ull << (ez & 63));
      hit = true;
      if (DISTINCT) {
        const uint32_t bit = 1u << (e & 31);
        const uint32_t old = atomicOr(&a.touch[(uint32_t)e >> 5], bit);
        dhit = !(old & bit);
      }
    }
  }

  const int64_t V = (int64_t)nx * ny * nz;
  uint32_t* touch_p = DISTINCT ? a.touch + ((V + 31) >> 5) : nullptr;
  const int32_t span_x = ny * nz, span_xw = nx * ny * nz, span_yw = ny * nz;
  bool active = ray && (rem[0] + rem[1] + rem[2] > 0);
  int n_pass = 0, n_dpass = 0;
  while (__any(active)) {
    // ---- aggregated pass of the current voxel
    const int addr = active ? sidx : -1;
    const int prev = __shfl_up(addr, 1);
    const bool head = active && (lane == 0 || prev != addr);
    const unsigned long long hb = __ballot(head);
    const unsigned long long ab = __ballot(active);
    if (head) {
      const unsigned long long bnd = hb | ~ab;
      const unsigned long long after = lane == 63 ? 0ull : (bnd >> (lane + 1));
      const int len = after ? __ffsll((long long)after) : 64 - lane;
      atomicAdd(&a.passes[addr], len);
      if (DISTINCT) {
        const uint32_t bit = 1u << (addr & 31);
        const uint32_t old = atomicOr(&touch_p[(uint32_t)addr >> 5], bit);
        n_dpass += !(old & bit);
      }
    }
    if (active) {
      n_pass++;
      // ---- choose the axes with the smallest crossing time
      const bool ax = rem[0] > 0, ay = rem[1] > 0, az = rem[2] > 0;
      bool mx = ax && (!ay || exy <= 0) && (!az || exz <= 0);
      bool my = ay && (!ax || exy >= 0) && (!az || eyz <= 0);
      bool mz = az && (!ax || exz >= 0) && (!ay || eyz >= 0);
      const bool up = (mx && sg[0] > 0) || (my && sg[1] > 0) || (mz && sg[2] > 0);
      if (up) {
        mx = mx && sg[0] > 0;
        my = my && sg[1] > 0;
        mz = mz && sg[2] > 0;
      }
      bool out = false;
      if (mx) {
        rem[0]--;
        out = out || room[0] == 0;
        room[0]--;
        exy += kxy;
        exz += kxz;
        sc[0] += sg[0];
        sidx += sg[0] * span_x;
        if (sc[0] == nx) { sc[0] = 0; sidx -= span_xw; }
        if (sc[0] < 0) { sc[0] = nx - 1; sidx += span_xw; }
      }
      if (my) {
        rem[1]--;
        out = out || room[1] == 0;
        room[1]--;
        exy -= kyx;
        eyz += kyz;
        sc[1] += sg[1];
        sidx += sg[1] * nz;
        if (sc[1] == ny) { sc[1] = 0; sidx -= span_yw; }
        if (sc[1] < 0) { sc[1] = ny - 1; sidx += span_yw; }
      }
      if (mz) {
        rem[2]--;
        out = out || room[2] == 0;
        room[2]--;
        exz -= kzx;
        eyz -= kzy;
        sc[2] += sg[2];
        sidx += sg[2];
        if (sc[2] == nz) { sc[2] = 0; sidx -= nz; }
        if (sc[2] < 0) { sc[2] = nz - 1; sidx += nz; }
      }
      active = !out && (rem[0] + rem[1] + rem[2] > 0);
    }
  }

  // ---- counters: one atomic per wave and counter
  const int c0 = __popcll(__ballot(nonfinite));
  const int c1 = __popcll(__ballot(outrange));
  const int c2 = __popcll(__ballot(hit));
  const int c3 = wave_sum(n_pass);
  if (lane == 0) {
    if (c0) atomicAdd(&a.stats[0], (unsigned long long)c0);
    if (c1) atomicAdd(&a.stats[1], (unsigned long long)c1);
    if (c2) atomicAdd(&a.stats[2], (unsigned long long)c2);
    if (c3) atomicAdd(&a.stats[3], (unsigned long long)c3);
  }
  if (DISTINCT) {
    const int c4 = wave_sum(n_dpass);
    const int c5 = __popcll(__ballot(dhit));
    if (lane == 0) {
      atomicAdd(&a.stats[4], (unsigned long long)c4);
      atomicAdd(&a.stats[5], (unsigned long long)c5);
    }
  }
}

// Resets the storage voxels whose coordinates lie in the box
// [x0, x0+cx) x [y0, y0+cy) x [z0, z0+cz), each taken modulo the axis size.
__global__ __launch_bounds__(kBlock) void k_clear_box(Dims d, int32_t* hits, int32_t* passes,
                                                      int32_t* minqz, int32_t x0, int32_t cx,
                                                      int32_t y0, int32_t cy, int32_t z0,
                                                      int32_t cz) {
  const uint32_t total = (uint32_t)cx * cy * cz;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    const uint32_t kz = i % (uint32_t)cz;
    const uint32_t t = i / (uint32_t)cz;
    const uint32_t ky = t % (uint32_t)cy;
    const uint32_t kx = t / (uint32_t)cy;
    const uint32_t sx = (x0 + kx) % (uint32_t)d.nx;
    const uint32_t sy = (y0 + ky) % (uint32_t)d.ny;
    const uint32_t sz = (z0 + kz) % (uint32_t)d.nz;
    const uint32_t e = (sx * d.ny + sy) * d.nz + sz;
    hits[e] = 0;
    passes[e] = 0;
    minqz[e] = INT32_MAX;
  }
}

// occ &= keep for the columns of the box [x0, x0+cx) x [y0, y0+cy) (mod n).
__global__ __launch_bounds__(kBlock) void k_clear_occ(Dims d, unsigned long long* occ,
                                                      int32_t x0, int32_t cx, int32_t y0,
                                                      int32_t cy, unsigned long long keep0,
                                                      unsigned long long keep1) {
  const uint32_t total = (uint32_t)cx * cy;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < total; i += gridDim.x * kBlock) {
    const uint32_t sx = (x0 + i / (uint32_t)cy) % (uint32_t)d.nx;
    const uint32_t sy = (y0 + i % (uint32_t)cy) % (uint32_t)d.ny;
    const uint32_t col = sx * d.ny + sy;
    occ[(size_t)col * d.W] &= keep0;
    if (d.W > 1) occ[(size_t)col * d.W + 1] &= keep1;
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_clear_box(const Dims& d, int32_t* hits, int32_t* passes, int32_t* minqz,
                            int32_t x0, int32_t cx, int32_t y0, int32_t cy, int32_t z0,
                            int32_t cz, hipStream_t s) {
  const int64_t total = (int64_t)cx * cy * cz;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_box, dim3(grid_for(total)), dim3(kBlock), 0, s, d, hits, passes,
                     minqz, x0, cx, y0, cy, z0, cz);
  return hipGetLastError();
}

hipError_t launch_clear_occ(const Dims& d, unsigned long long* occ, int32_t x0, int32_t cx,
                            int32_t y0, int32_t cy, unsigned long long keep0,
                            unsigned long long keep1, hipStream_t s) {
  const int64_t total = (int64_t)cx * cy;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_occ, dim3(grid_for(total)), dim3(kBlock), 0, s, d, occ, x0, cx,
                     y0, cy, keep0, keep1);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_insert(const InsertArgs& a, bool distinct, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int g = (a.n + kBlock - 1) / kBlock;
  if (distinct)
    hipLaunchKernelGGL(k_insert<true>, dim3(g), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_insert<false>, dim3(g), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace gvom
