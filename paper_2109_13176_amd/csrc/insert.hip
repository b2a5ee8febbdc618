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

// ---------------------------------------------------------------------------
// Pass 1, one lane per point: transform, record the return in its voxel, and
// cut the ray into segments for the traversal pass.
//
// A ray's voxel path is monotone in every axis.  Along its dominant axis (the
// axis with the most voxel steps) the path is cut every seg_len voxels:
// segment j holds the path voxels whose dominant coordinate lies j*seg_len ..
// (j+1)*seg_len - 1 voxels from the sensor's.  Only segments that start
// inside the window along the dominant axis are emitted.  A wave reserves
// room for all its segments with one atomic and writes them segment-major,
// so that consecutive items are the same segment of neighbouring rays.
__device__ __forceinline__ int dominant_axis(const int32_t n[3]) {
  return (n[1] > n[0]) ? (n[2] > n[1] ? 2 : 1) : (n[2] > n[0] ? 2 : 0);
}

// Transform of point i (in firing order) and its return: q = Q16 world
// coordinates; records the hit when the return lies in the window.  Returns
// true when the ray can be traversed.
struct PointFlags {
  bool nonfinite = false, outrange = false, hit = false, dhit = false;
};

template <bool DISTINCT>
__device__ __forceinline__ bool point_pass(const InsertArgs& a, const int i, int32_t q[3],
                                           PointFlags& f) {
  q[0] = q[1] = q[2] = 0;
  if (i >= a.n) return false;
  int pidx = i;
  if (a.fw > 1) {
    const int b = i / a.azimuths;
    pidx = (i - b * a.azimuths) * a.fw + b;
  }
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  const float p0 = a.xyz[3 * pidx + 0];
  const float p1 = a.xyz[3 * pidx + 1];
  const float p2 = a.xyz[3 * pidx + 2];
  if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) {
    f.nonfinite = true;
    return false;
  }
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
  if (!ok) {
    f.outrange = true;
    return false;
  }
  int32_t l[3];
  bool win = true;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    l[k] = (q[k] >> 16) - a.O[k];
    win = win && l[k] >= 0 && l[k] < dims[k];
  }
  if (win) {  // the return
    const int32_t ex = wrap_add(l[0] + a.d.ro[0], dims[0]);
    const int32_t ey = wrap_add(l[1] + a.d.ro[1], dims[1]);
    const int32_t ez = wrap_add(l[2] + a.d.ro[2], dims[2]);
    const int32_t col = ex * dims[1] + ey;
    const int32_t e = col_base(a.d, ex, ey) + (ez << 4);
    atomicAdd(&a.hits[e], 1);
    // min and or only move one way: a plain read that already satisfies
    // the update makes the atomic unnecessary
    if (q[2] < a.minqz[e]) atomicMin(&a.minqz[e], q[2]);
    unsigned long long* ow = &a.occ[(int64_t)col * a.d.W + (ez >> 6)];
    const unsigned long long ob = 1ull << (ez & 63);
    if (!(*ow & ob)) atomicOr(ow, ob);
    f.hit = true;
    if (DISTINCT) {
      const uint32_t bit = 1u << (e & 31);
      const uint32_t old = atomicOr(&a.touch[(uint32_t)e >> 5], bit);
      f.dhit = !(old & bit);
    }
  }
  return true;
}

template <bool DISTINCT>
__device__ __forceinline__ void rays_body(const InsertArgs& a, const int blk) {
  __shared__ unsigned int wcount[kRayBlock / 64][5];
  __shared__ unsigned long long wbase[kRayBlock / 64];
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int i = blk * kRayBlock + threadIdx.x;
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  int32_t q[3];
  PointFlags pf;
  const bool ray = point_pass<DISTINCT>(a, i, q, pf);
  const bool nonfinite = pf.nonfinite, outrange = pf.outrange, hit = pf.hit, dhit = pf.dhit;

  int nseg = 0;
  if (ray) {
    int32_t n[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int32_t sv = a.S[k] >> 16, ev = q[k] >> 16;
      n[k] = ev > sv ? ev - sv : sv - ev;
    }
    if (n[0] + n[1] + n[2] > 0) {
      const int dom = dominant_axis(n);
      const int32_t sv = a.S[dom] >> 16;
      const int32_t lc = sv - a.O[dom];
      const int32_t room = q[dom] > a.S[dom] ? dims[dom] - 1 - lc : lc;
      nseg = min(n[dom], room) / a.seg_len + 1;
    }
  }

  // reserve and write the segments, segment-major within the wave: one
  // returning atomic per block, wave bases from the block's prefix
  int total = nseg;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o);
  int maxseg = nseg;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) maxseg = max(maxseg, __shfl_xor(maxseg, o));
  const int c0 = __popcll(__ballot(nonfinite));
  const int c1 = __popcll(__ballot(outrange));
  const int c2 = __popcll(__ballot(hit));
  const int c5 = DISTINCT ? __popcll(__ballot(dhit)) : 0;
  if (lane == 0) {
    wcount[wv][0] = total;
    wcount[wv][1] = c0;
    wcount[wv][2] = c1;
    wcount[wv][3] = c2;
    wcount[wv][4] = c5;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum = 0, s0 = 0, s1 = 0, s2 = 0, s5 = 0;
    for (int w = 0; w < kRayBlock / 64; w++) {
      wbase[w] = sum;
      sum += wcount[w][0];
      s0 += wcount[w][1];
      s1 += wcount[w][2];
      s2 += wcount[w][3];
      s5 += wcount[w][4];
    }
    // blocks are spread over kStripes counters, each with its own item region
    const int st = blk % kStripes;
    const unsigned long long b = sum ? atomicAdd(&a.stats[8 + st], sum) : 0ull;
    for (int w = 0; w < kRayBlock / 64; w++) wbase[w] += b + a.stripe_off[st];
    unsigned long long* pr = a.part_rays + 4 * (size_t)blk;
    pr[0] = s0;
    pr[1] = s1;
    pr[2] = s2;
    pr[3] = s5;
  }
  __syncthreads();
  unsigned long long off = wbase[wv];
  for (int j = 0; j < maxseg; j++) {
    const unsigned long long m = __ballot(nseg > j);
    if (nseg > j) {
      const unsigned long long pos =
          off + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      a.items[pos] = make_int4(q[0], q[1], q[2], j);
    }
    off += __popcll(m);
  }
}

template <bool DISTINCT>
__global__ __launch_bounds__(kRayBlock) void k_rays(InsertArgs a) {
  rays_body<DISTINCT>(a, blockIdx.x);
}

// floor(x / d) for d > 0 (|x| < 2^60): double estimate, exact integer fix-up.
__device__ __forceinline__ int64_t floor_div_pos(int64_t x, int64_t d, bool* exact) {
  int64_t q = (int64_t)floor((double)x / (double)d);
  int64_t r = x - q * d;
  while (r < 0) { q--; r += d; }
  while (r >= d) { q++; r -= d; }
  *exact = r == 0;
  return q;
}

// ---------------------------------------------------------------------------
// Pass 2, one lane per ray segment: walk the segment voxel by voxel and add
// one pass to every window voxel before the ray's end voxel.
//
// Start voxel of segment j > 0: the instant the dominant axis enters cell
// c = c_sensor +- j*seg_len, at exact time t = num / |D_dom|.  Another axis b
// then lies in cell floor(X_b(t)); if X_b(t) is exactly on a boundary while
// both b and the dominant axis move down, b leaves its cell at the same
// instant as the dominant axis (one cell lower).
//
// Traversal: along axis a the segment leaves its current cell when it has
// moved num_a (Q units) at speed |D_a|, i.e. at time num_a / |D_a|.  The axis
// with the smallest time steps next; times are compared exactly through the
// pairwise differences E_ab = num_a |D_b| - num_b |D_a| (int64, |.| < 2^56),
// which change by constant increments when an axis steps.  When several axes
// share the smallest time, the axes moving up step first (the shared boundary
// belongs to the upper cell) and the axes moving down step in the next
// iteration, so the voxel at that instant is visited.
//
// Lanes of a wave step in lock-step; the lanes that pass the same voxel as
// their left neighbour join its run and the run's first lane adds the run
// length with one atomic.
template <bool DISTINCT>
__device__ __forceinline__ void trace_body(const InsertArgs& a, const int blk, const int nblk) {
  const int lane = __lane_id();
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int32_t dims[3] = {nx, ny, nz};
  // items of stripe t occupy [stripe_off[t], stripe_off[t] + cnt[t]); the
  // loop runs over their concatenation
  int64_t pre[kStripes + 1];
  pre[0] = 0;
#pragma unroll
  for (int t = 0; t < kStripes; t++)
    pre[t + 1] = pre[t] + min((int64_t)a.stats[8 + t], a.stripe_cap[t]);
  const int64_t count = pre[kStripes];
  const int64_t stride = (int64_t)nblk * kBlock;
  uint32_t* touch_p = DISTINCT ? a.touch + ((a.d.vs + 31) >> 5) : nullptr;
  int n_pass = 0, n_dpass = 0;

  for (int64_t wbase = (int64_t)blk * kBlock + (threadIdx.x & ~63); wbase < count;
       wbase += stride) {
    const int64_t it = wbase + lane;
    bool active = false;
    int32_t rem[3] = {0, 0, 0}, room[3] = {0, 0, 0}, sg[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
    int64_t exy = 0, exz = 0, eyz = 0;
    int64_t kxy = 0, kxz = 0, kyx = 0, kyz = 0, kzx = 0, kzy = 0;
    int32_t sidx = 0, segleft = 0;
    bool mdx = false, mdy = false, mdz = false;
    if (it < count) {
      int t = 0;
#pragma unroll
      for (int k = 1; k < kStripes; k++) t += it >= pre[k];
      const int4 item = a.items[a.stripe_off[t] + (it - pre[t])];
      const int32_t q[3] = {item.x, item.y, item.z};
      const int j = item.w;
      int32_t sv[3], ev[3], n[3], ad[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        sv[k] = a.S[k] >> 16;
        ev[k] = q[k] >> 16;
        n[k] = ev[k] > sv[k] ? ev[k] - sv[k] : sv[k] - ev[k];
        const int32_t dq = q[k] - a.S[k];
        sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
        ad[k] = dq < 0 ? -dq : dq;
      }
      const int dom = dominant_axis(n);
      int32_t v[3] = {sv[0], sv[1], sv[2]};
      if (j > 0) {
        const int32_t c = sv[dom] + sg[dom] * j * a.seg_len;
        const int64_t num = sg[dom] > 0 ? ((int64_t)c << 16) - a.S[dom]
                                        : (int64_t)a.S[dom] - (((int64_t)c + 1) << 16);
        const int64_t den = (int64_t)ad[dom] << 16;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          if (k == dom) {
            v[k] = c;
            continue;
          }
          bool exact;
          const int64_t x = (int64_t)a.S[k] * ad[dom] + num * (sg[k] * (int64_t)ad[k]);
          int64_t vb = floor_div_pos(x, den, &exact);
          if (exact && sg[dom] < 0 && sg[k] < 0) vb -= 1;
          v[k] = (int32_t)vb;
        }
      }
      bool inside = true;
      int32_t l[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        l[k] = v[k] - a.O[k];
        inside = inside && l[k] >= 0 && l[k] < dims[k];
      }
      if (inside) {
        int64_t num[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
          rem[k] = ev[k] > v[k] ? ev[k] - v[k] : v[k] - ev[k];
          room[k] = sg[k] > 0 ? dims[k] - 1 - l[k] : l[k];
          num[k] = sg[k] > 0 ? (((int64_t)v[k] + 1) << 16) - a.S[k]
                             : (int64_t)a.S[k] - ((int64_t)v[k] << 16);
          sc[k] = wrap_add(l[k] + a.d.ro[k], dims[k]);
        }
        exy = num[0] * ad[1] - num[1] * ad[0];
        exz = num[0] * ad[2] - num[2] * ad[0];
        eyz = num[1] * ad[2] - num[2] * ad[1];
        kxy = (int64_t)ad[1] << 16;
        kxz = (int64_t)ad[2] << 16;
        kyx = (int64_t)ad[0] << 16;
        kyz = (int64_t)ad[2] << 16;
        kzx = (int64_t)ad[0] << 16;
        kzy = (int64_t)ad[1] << 16;
        sidx = col_base(a.d, sc[0], sc[1]) + (sc[2] << 4);
        segleft = a.seg_len - 1;
        mdx = dom == 0;
        mdy = dom == 1;
        mdz = dom == 2;
        active = rem[0] + rem[1] + rem[2] > 0;
      }
    }

    // per-lane constants of the branch-free step
    const bool px = sg[0] > 0, py = sg[1] > 0, pz = sg[2] > 0;
    const int32_t trig0 = px ? nx : -1, trig1 = py ? ny : -1, trig2 = pz ? nz : -1;
    const int32_t wv0 = px ? 0 : nx - 1, wv1 = py ? 0 : ny - 1, wv2 = pz ? 0 : nz - 1;
    while (__any(active)) {
      // ---- aggregated pass of the current voxel: runs of equal addresses in
      // neighbouring lanes (left neighbour via a whole-wave DPP shift)
      const int addr = active ? sidx : -1;
      const int prev = __builtin_amdgcn_update_dpp(-2, addr, 0x138, 0xf, 0xf, false);
      const bool head = active && prev != addr;
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
      n_pass += active;
      // ---- the axes with the smallest crossing time (branch-free)
      const bool ax = rem[0] > 0, ay = rem[1] > 0, az = rem[2] > 0;
      bool mx = ax & (!ay | (exy <= 0)) & (!az | (exz <= 0));
      bool my = ay & (!ax | (exy >= 0)) & (!az | (eyz <= 0));
      bool mz = az & (!ax | (exz >= 0)) & (!ay | (eyz >= 0));
      const bool up = (mx & px) | (my & py) | (mz & pz);
      mx = mx & (!up | px);
      my = my & (!up | py);
      mz = mz & (!up | pz);
      const bool domstep = (mx & mdx) | (my & mdy) | (mz & mdz);
      const bool out = (domstep & (segleft == 0)) | (mx & (room[0] == 0)) |
                       (my & (room[1] == 0)) | (mz & (room[2] == 0));
      segleft -= domstep;
      rem[0] -= mx;
      rem[1] -= my;
      rem[2] -= mz;
      room[0] -= mx;
      room[1] -= my;
      room[2] -= mz;
      exy += (mx ? kxy : 0) - (my ? kyx : 0);
      exz += (mx ? kxz : 0) - (mz ? kzx : 0);
      eyz += (my ? kyz : 0) - (mz ? kzy : 0);
      const int32_t t0 = sc[0] + (mx ? sg[0] : 0);
      const int32_t t1 = sc[1] + (my ? sg[1] : 0);
      const int32_t t2 = sc[2] + (mz ? sg[2] : 0);
      const bool w0 = t0 == trig0, w1 = t1 == trig1, w2 = t2 == trig2;
      sc[0] = w0 ? wv0 : t0;
      sc[1] = w1 ? wv1 : t1;
      sc[2] = w2 ? wv2 : t2;
      sidx = col_base(a.d, sc[0], sc[1]) + (sc[2] << 4);
      active = active & !out & (rem[0] + rem[1] + rem[2] > 0);
    }
  }

  // per-block counters, written without atomics (summed by the host)
  __shared__ int wsum[kBlock / 64][2];
  const int c3 = wave_sum(n_pass);
  const int c4 = DISTINCT ? wave_sum(n_dpass) : 0;
  if (lane == 0) {
    wsum[threadIdx.x >> 6][0] = c3;
    wsum[threadIdx.x >> 6][1] = c4;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long p = 0, q = 0;
    for (int w = 0; w < kBlock / 64; w++) {
      p += wsum[w][0];
      q += wsum[w][1];
    }
    a.part_trace[2 * blk] = p;
    a.part_trace[2 * blk + 1] = q;
  }
}

template <bool DISTINCT>
__global__ __launch_bounds__(kBlock) void k_trace(InsertArgs a) {
  trace_body<DISTINCT>(a, blockIdx.x, gridDim.x);
}

// Window scroll: box k resets the storage voxels of
// [x0, x0+cx) x [y0, y0+cy) x [z0, z0+cz) (each coordinate modulo the axis
// size).  Occupancy: a box spanning all z (an x or y slab) zeroes the words
// of its columns; a z slab (spanning all columns) clears its bits in every
// column, where one thread combines all boxes of the column so that no two
// threads update one word.
__device__ __forceinline__ void clear_body(const ClearArgs& a, const int64_t first,
                                           const int64_t stride) {
  const Dims& d = a.d;
  bool zslab = false;
  for (int k = 0; k < a.nbox; k++) {
    const int32_t* bx = a.box[k];
    const uint32_t cx = bx[1], cy = bx[3], cz = bx[5];
    zslab = zslab || (int)cz < d.nz;
    const uint32_t total = cx * cy * cz;
    for (int64_t i = first; i < total; i += stride) {
      const uint32_t kz = (uint32_t)i % cz;
      const uint32_t t = (uint32_t)i / cz;
      const uint32_t ky = t % cy;
      const uint32_t kx = t / cy;
      const uint32_t sx = (bx[0] + kx) % (uint32_t)d.nx;
      const uint32_t sy = (bx[2] + ky) % (uint32_t)d.ny;
      const uint32_t sz = (bx[4] + kz) % (uint32_t)d.nz;
      const uint32_t e = (uint32_t)col_base(d, sx, sy) + (sz << 4);
      a.hits[e] = 0;
      a.passes[e] = 0;
      a.minqz[e] = INT32_MAX;
    }
  }
  if (!zslab) {
    for (int k = 0; k < a.nbox; k++) {
      const int32_t* bx = a.box[k];
      const uint32_t cx = bx[1], cy = bx[3];
      for (int64_t i = first; i < (int64_t)cx * cy; i += stride) {
        const uint32_t sx = (bx[0] + (uint32_t)i / cy) % (uint32_t)d.nx;
        const uint32_t sy = (bx[2] + (uint32_t)i % cy) % (uint32_t)d.ny;
        const uint32_t col = sx * d.ny + sy;
        a.occ[(size_t)col * d.W] = 0;
        if (d.W > 1) a.occ[(size_t)col * d.W + 1] = 0;
      }
    }
  } else {
    for (int64_t i = first; i < (int64_t)d.nx * d.ny; i += stride) {
      const uint32_t sx = (uint32_t)i / d.ny, sy = (uint32_t)i % d.ny;
      unsigned long long k0 = ~0ull, k1 = ~0ull;
      for (int k = 0; k < a.nbox; k++) {
        const int32_t* bx = a.box[k];
        const uint32_t rx = (sx + d.nx - bx[0]) % (uint32_t)d.nx;
        const uint32_t ry = (sy + d.ny - bx[2]) % (uint32_t)d.ny;
        if (rx < (uint32_t)bx[1] && ry < (uint32_t)bx[3]) {
          k0 &= a.keep[k][0];
          k1 &= a.keep[k][1];
        }
      }
      a.occ[(size_t)i * d.W] &= k0;
      if (d.W > 1) a.occ[(size_t)i * d.W + 1] &= k1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_clear(ClearArgs a) {
  clear_body(a, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock);
}

// ---------------------------------------------------------------------------
// Binned traversal.
//
// Storage columns are cut into slabs of kBinT cells along x and along y.  A
// ray whose dominant axis d is x or y is cut where its storage coordinate
// along d enters a new slab, so every piece (segment) lies in one slab.  A
// segment is binned by d, the direction of its cross axis c, its slab g and
// the kBinT-tile h of its start's storage c coordinate.  The bin's region is
// the slab x kBinRows storage rows along c from the tile towards the side the
// ray moves to x all z levels; it holds every voxel of the segment except, at
// most, a few of a short steep ray, which go to global memory directly.
// A persistent work group takes one unit (up to kUnit segments of one bin)
// at a time, counts the unit's passes in 16-bit LDS counters laid out like
// the storage bricks, then adds the counters of the touched z levels to the
// passes array with coalesced atomics (regions of different units overlap).
// Rays whose dominant axis is z go to the last bin; they are cut every kSegG
// cells from the sensor and traced with global atomics.

// Voxel at which the ray S -> q enters world cell c along axis dm (c is not
// the sensor's cell): see the traversal pass below for the tie rule.
__device__ __forceinline__ void entry_voxel(const int32_t S[3], const int32_t sg[3],
                                            const int32_t ad[3], const int dm, const int32_t c,
                                            int32_t v[3]) {
  const int64_t num = sg[dm] > 0 ? ((int64_t)c << 16) - S[dm] : (int64_t)S[dm] - (((int64_t)c + 1) << 16);
  const int64_t den = (int64_t)ad[dm] << 16;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    if (k == dm) {
      v[k] = c;
      continue;
    }
    bool exact;
    const int64_t x = (int64_t)S[k] * ad[dm] + num * (sg[k] * (int64_t)ad[k]);
    int64_t vb = floor_div_pos(x, den, &exact);
    if (exact && sg[dm] < 0 && sg[k] < 0) vb -= 1;
    v[k] = (int32_t)vb;
  }
}

// Calls emit(bin, word) for every segment of the ray S -> q that starts in
// the window.  Binned segment: word = d offset in the slab | cross offset in
// the region << 4 | storage z << 10.  Z-dominant ray: bin nb - 1, word =
// segment index.
template <class F>
__device__ __forceinline__ void for_segments(const InsertArgs& a, const int32_t q[3], F&& emit) {
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  int32_t sv[3], ev[3], n[3], sg[3], ad[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    sv[k] = a.S[k] >> 16;
    ev[k] = q[k] >> 16;
    n[k] = ev[k] > sv[k] ? ev[k] - sv[k] : sv[k] - ev[k];
    const int32_t dq = q[k] - a.S[k];
    sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
    ad[k] = dq < 0 ? -dq : dq;
  }
  if (n[0] + n[1] + n[2] == 0) return;
  const int dom = dominant_axis(n);
  if (dom == 2) {
    const int32_t lc = sv[2] - a.O[2];
    const int32_t room = sg[2] > 0 ? dims[2] - 1 - lc : lc;
    const int nseg = min(n[2], room) / kSegG + 1;
    for (int j = 0; j < nseg; j++) emit(a.nb - 1, j);
    return;
  }
  const int d = dom, c = 1 - dom;
  const int32_t nd = dims[d], nc = dims[c];
  const bool cneg = sg[c] < 0;
  const int base = (d == 0 ? 0 : 2 * a.gx * a.gy) + (cneg ? a.gx * a.gy : 0);
  const int ntile = d == 0 ? a.gy : a.gx;
  const int32_t led = ev[d] - a.O[d];
  const int32_t last = sg[d] > 0 ? min(led, nd - 1) : max(led, 0);
  int32_t ld = sv[d] - a.O[d];
  bool first = true;
  while (sg[d] > 0 ? ld <= last : ld >= last) {
    int32_t v[3] = {sv[0], sv[1], sv[2]};
    if (!first) entry_voxel(a.S, sg, ad, d, a.O[d] + ld, v);
    first = false;
    int32_t l[3];
    bool inside = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      l[k] = v[k] - a.O[k];
      inside = inside && l[k] >= 0 && l[k] < dims[k];
    }
    if (!inside) break;  // monotone path: it does not come back
    const int32_t sd = wrap_add(l[d] + a.d.ro[d], nd);
    const int32_t scc = wrap_add(l[c] + a.d.ro[c], nc);
    const int32_t sz = wrap_add(l[2] + a.d.ro[2], dims[2]);
    const int g = sd / kBinT, h = scc / kBinT;
    const int doff = sd - g * kBinT;
    const int coff = scc - h * kBinT + (cneg ? kBinRows - kBinT : 0);
    emit(base + g * ntile + h, doff | (coff << 4) | (sz << 10));
    if (sg[d] > 0)
      ld += min(g * kBinT + kBinT, nd) - sd;
    else
      ld -= doff + 1;
  }
}

// One lane per point: transform and return as in the segmented pass, then
// the ray's segments are counted per bin (LDS), the block reserves item room
// and publishes one entry {first item, count} per non-empty bin, and the
// segments are enumerated again and written bin by bin.
template <bool DISTINCT>
__global__ __launch_bounds__(kRayBlock) void k_rays_bin(InsertArgs a) {
  extern __shared__ int hist[];  // a.nb counters, then exclusive offsets
  __shared__ unsigned int wcount[kRayBlock / 64][4];
  __shared__ int wtot[kRayBlock / 64];
  __shared__ long long s_base;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int blk = blockIdx.x;
  for (int i = threadIdx.x; i < a.nb; i += kRayBlock) hist[i] = 0;
  int32_t q[3];
  PointFlags pf;
  const bool ray = point_pass<DISTINCT>(a, blk * kRayBlock + threadIdx.x, q, pf);
  const int c0 = __popcll(__ballot(pf.nonfinite));
  const int c1 = __popcll(__ballot(pf.outrange));
  const int c2 = __popcll(__ballot(pf.hit));
  const int c5 = DISTINCT ? __popcll(__ballot(pf.dhit)) : 0;
  if (lane == 0) {
    wcount[wv][0] = c0;
    wcount[wv][1] = c1;
    wcount[wv][2] = c2;
    wcount[wv][3] = c5;
  }
  __syncthreads();
  if (ray) for_segments(a, q, [&](int bin, int) { atomicAdd(&hist[bin], 1); });
  __syncthreads();
  // block-wide exclusive scan of the bin counts (contiguous chunk per thread)
  const int per = (a.nb + kRayBlock - 1) / kRayBlock;
  const int i0 = threadIdx.x * per;
  int s = 0;
  for (int k = 0; k < per && i0 + k < a.nb; k++) s += hist[i0 + k];
  int incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    unsigned long long s0 = 0, s1 = 0, s2 = 0, s5 = 0;
    for (int w = 0; w < kRayBlock / 64; w++) {
      const int t = wtot[w];
      wtot[w] = sum;
      sum += t;
      s0 += wcount[w][0];
      s1 += wcount[w][1];
      s2 += wcount[w][2];
      s5 += wcount[w][3];
    }
    const int st = blk % kStripes;
    const unsigned long long b = sum ? atomicAdd(&a.stats[8 + st], (unsigned long long)sum) : 0ull;
    s_base = (long long)(a.stripe_off[st] + (int64_t)b);
    unsigned long long* pr = a.part_rays + 4 * (size_t)blk;
    pr[0] = s0;
    pr[1] = s1;
    pr[2] = s2;
    pr[3] = s5;
  }
  __syncthreads();
  const long long base = s_base;
  int off = wtot[wv] + incl - s;
  for (int k = 0; k < per && i0 + k < a.nb; k++) {
    const int bin = i0 + k;
    const int cnt = hist[bin];
    hist[bin] = off;
    if (cnt) {
      const int slot = atomicAdd(&a.bin_nent[bin], 1);
      a.bin_ent[(int64_t)bin * a.maxblk + slot] = make_int2((int)(base + off), cnt);
      atomicAdd(&a.bin_tot[bin], cnt);
    }
    off += cnt;
  }
  __syncthreads();
  if (ray)
    for_segments(a, q, [&](int bin, int w) {
      const int pos = atomicAdd(&hist[bin], 1);
      a.items[base + pos] = make_int4(q[0], q[1], q[2], w);
    });
}

// One block: the work units of every bin (full units first, so that the
// long ones start early), the entry counts the traversal reads, and the bin
// counters cleared for the next scan.
__global__ __launch_bounds__(1024) void k_binscan(InsertArgs a) {
  __shared__ int wt[2][16];
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int per = (a.nb + 1023) / 1024;
  const int i0 = threadIdx.x * per;
  int nf = 0, np = 0;
  for (int k = 0; k < per && i0 + k < a.nb; k++) {
    const int t = a.bin_tot[i0 + k];
    nf += t / kUnit;
    np += (t % kUnit) != 0;
  }
  int f = nf, p = np;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int uf = __shfl_up(f, o), up = __shfl_up(p, o);
    if (lane >= o) {
      f += uf;
      p += up;
    }
  }
  if (lane == 63) {
    wt[0][wv] = f;
    wt[1][wv] = p;
  }
  __syncthreads();
  int bf = 0, bp = 0, F = 0, P = 0;
  for (int w = 0; w < 16; w++) {
    if (w < wv) {
      bf += wt[0][w];
      bp += wt[1][w];
    }
    F += wt[0][w];
    P += wt[1][w];
  }
  int uf = bf + f - nf, up = F + bp + p - np;
  for (int k = 0; k < per && i0 + k < a.nb; k++) {
    const int bin = i0 + k;
    const int t = a.bin_tot[bin];
    const int full = t / kUnit;
    for (int j = 0; j < full; j++) a.units[uf++] = make_int4(bin, j * kUnit, kUnit, 0);
    if (t % kUnit) a.units[up++] = make_int4(bin, full * kUnit, t % kUnit, 0);
    a.bin_snap[bin] = a.bin_nent[bin];
    a.bin_nent[bin] = 0;
    a.bin_tot[bin] = 0;
  }
  if (threadIdx.x == 0) {
    a.uctl[0] = F + P;
    a.uctl[1] = 0;
  }
}

__device__ __forceinline__ int32_t mod_pos(int32_t v, int32_t n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Adds one pass to storage voxel e (global memory), with its distinct bit.
template <bool DISTINCT>
__device__ __forceinline__ void global_pass(const InsertArgs& a, uint32_t* touch_p, int32_t e,
                                            int32_t cnt, int& n_dpass) {
  atomicAdd(&a.passes[e], cnt);
  if (DISTINCT) {
    const uint32_t bit = 1u << (e & 31);
    const uint32_t old = atomicOr(&touch_p[(uint32_t)e >> 5], bit);
    n_dpass += !(old & bit);
  }
}

// Exact traversal state of one segment: remaining steps to the end voxel and
// to the window edge per axis, crossing-time differences, step constants.
struct Walk {
  int32_t rem[3], room[3], sg[3];
  int64_t exy, exz, eyz, kx, ky, kz;  // k*: |D| << 16 per axis
};

// Starts the walk at world voxel v (inside the window, local l).
__device__ __forceinline__ void walk_init(const InsertArgs& a, const int32_t q[3],
                                          const int32_t v[3], const int32_t l[3], Walk& w) {
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  int64_t num[3];
  int32_t ad[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const int32_t ev = q[k] >> 16;
    const int32_t dq = q[k] - a.S[k];
    w.sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
    ad[k] = dq < 0 ? -dq : dq;
    w.rem[k] = ev > v[k] ? ev - v[k] : v[k] - ev;
    w.room[k] = w.sg[k] > 0 ? dims[k] - 1 - l[k] : l[k];
    num[k] = w.sg[k] > 0 ? (((int64_t)v[k] + 1) << 16) - a.S[k] : (int64_t)a.S[k] - ((int64_t)v[k] << 16);
  }
  w.exy = num[0] * ad[1] - num[1] * ad[0];
  w.exz = num[0] * ad[2] - num[2] * ad[0];
  w.eyz = num[1] * ad[2] - num[2] * ad[1];
  w.kx = (int64_t)ad[0] << 16;
  w.ky = (int64_t)ad[1] << 16;
  w.kz = (int64_t)ad[2] << 16;
}

// One step: the axes with the smallest crossing time (ties: axes moving up
// first), see the segmented traversal pass.  Sets mx/my/mz; returns whether
// an axis left the window.
__device__ __forceinline__ bool walk_step(Walk& w, bool& mx, bool& my, bool& mz) {
  const bool ax = w.rem[0] > 0, ay = w.rem[1] > 0, az = w.rem[2] > 0;
  const bool px = w.sg[0] > 0, py = w.sg[1] > 0, pz = w.sg[2] > 0;
  mx = ax & (!ay | (w.exy <= 0)) & (!az | (w.exz <= 0));
  my = ay & (!ax | (w.exy >= 0)) & (!az | (w.eyz <= 0));
  mz = az & (!ax | (w.exz >= 0)) & (!ay | (w.eyz >= 0));
  const bool up = (mx & px) | (my & py) | (mz & pz);
  mx = mx & (!up | px);
  my = my & (!up | py);
  mz = mz & (!up | pz);
  const bool out = (mx & (w.room[0] == 0)) | (my & (w.room[1] == 0)) | (mz & (w.room[2] == 0));
  w.rem[0] -= mx;
  w.rem[1] -= my;
  w.rem[2] -= mz;
  w.room[0] -= mx;
  w.room[1] -= my;
  w.room[2] -= mz;
  w.exy += (mx ? w.ky : 0) - (my ? w.kx : 0);
  w.exz += (mx ? w.kz : 0) - (mz ? w.kx : 0);
  w.eyz += (my ? w.kz : 0) - (mz ? w.ky : 0);
  return out;
}

// Sets the storage levels (lo + k) mod nz, k = 0..len-1 (lo < nz, len <= nz + 1),
// in the 128-bit mask m0 | m1 << 64.
__device__ __forceinline__ void mark_levels(unsigned long long& m0, unsigned long long& m1, int lo,
                                            int len, int nz) {
  for (int k = 0; k < len; k++) {
    int z = lo + k;
    z = z >= nz ? z - nz : z;
    const unsigned long long bit = 1ull << (z & 63);
    if (z < 64) m0 |= bit; else m1 |= bit;
  }
}

template <bool DISTINCT>
__global__ __launch_bounds__(kTraceBinThreads) void k_trace_bin(InsertArgs a) {
  extern __shared__ uint32_t cnt[];  // kLevelWords per storage z level
  __shared__ int s_eoff[kMaxEnt];
  __shared__ int s_epre[kMaxEnt + 1];
  __shared__ int4 s_unit;
  __shared__ unsigned long long s_lev[2];
  __shared__ int s_levlist[128];
  __shared__ int s_nlev;
  __shared__ int wtot[kTraceBinThreads / 64];
  __shared__ int wsum[kTraceBinThreads / 64][2];
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int32_t dims[3] = {nx, ny, nz};
  for (int i = tid; i < kLevelWords * nz; i += kTraceBinThreads) cnt[i] = 0;
  if (tid == 0) {
    s_lev[0] = 0;
    s_lev[1] = 0;
  }
  uint32_t* touch_p = DISTINCT ? a.touch + ((a.d.vs + 31) >> 5) : nullptr;
  int n_pass = 0, n_dpass = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) {
      const int u = atomicAdd(&a.uctl[1], 1);
      s_unit = u < a.uctl[0] ? a.units[u] : make_int4(-1, 0, 0, 0);
    }
    __syncthreads();
    const int4 un = s_unit;
    if (un.x < 0) break;
    const int bin = un.x;
    const int nent = a.bin_snap[bin];
    // entries of the bin and their exclusive prefix (one per thread)
    int ec = 0;
    if (tid < nent) {
      const int2 e = a.bin_ent[(int64_t)bin * a.maxblk + tid];
      s_eoff[tid] = e.x;
      ec = e.y;
    }
    int incl = ec;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    int wb = 0;
    for (int w = 0; w < wv; w++) wb += wtot[w];
    if (tid < nent) s_epre[tid] = wb + incl - ec;
    __syncthreads();

    const bool glob = bin == a.nb - 1;
    // region of the bin
    int d = 0, g = 0, h = 0;
    bool cneg = false;
    if (!glob) {
      const int half = a.gx * a.gy;
      int r = bin;
      if (r >= 2 * half) {
        d = 1;
        r -= 2 * half;
      }
      cneg = r >= half;
      r -= cneg ? half : 0;
      const int ntile = d == 0 ? a.gy : a.gx;
      g = r / ntile;
      h = r - g * ntile;
    }
    const int32_t nd = d == 0 ? nx : ny, nc = d == 0 ? ny : nx;
    const int32_t rod = d == 0 ? a.d.ro[0] : a.d.ro[1], roc = d == 0 ? a.d.ro[1] : a.d.ro[0];
    const int32_t rd0 = g * kBinT;
    const int32_t rc0 = h * kBinT - (cneg ? kBinRows - kBinT : 0);
    const int nbyr = d == 0 ? kBinRows / 4 : kBinT / 4;  // bricks along y in the region
    const int32_t rx0 = d == 0 ? rd0 : rc0, ry0 = d == 0 ? rc0 : rd0;
    unsigned long long lev0 = 0ull, lev1 = 0ull;

    for (int vi = un.y + tid; vi < un.y + un.z; vi += kTraceBinThreads) {
      int lo = 0, hi = nent;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_epre[mid] <= vi) lo = mid; else hi = mid;
      }
      const int4 item = a.items[s_eoff[lo] + (vi - s_epre[lo])];
      const int32_t q[3] = {item.x, item.y, item.z};
      if (glob) {
        // z-dominant ray: segment item.w of kSegG cells from the sensor
        int32_t sg[3], ad[3], sv[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
          sv[k] = a.S[k] >> 16;
          const int32_t dq = q[k] - a.S[k];
          sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
          ad[k] = dq < 0 ? -dq : dq;
        }
        int32_t v[3] = {sv[0], sv[1], sv[2]};
        if (item.w > 0) entry_voxel(a.S, sg, ad, 2, sv[2] + sg[2] * item.w * kSegG, v);
        int32_t l[3];
        bool inside = true;
#pragma unroll
        for (int k = 0; k < 3; k++) {
          l[k] = v[k] - a.O[k];
          inside = inside && l[k] >= 0 && l[k] < dims[k];
        }
        if (!inside) continue;
        Walk w;
        walk_init(a, q, v, l, w);
        int32_t sc[3];
#pragma unroll
        for (int k = 0; k < 3; k++) sc[k] = wrap_add(l[k] + a.d.ro[k], dims[k]);
        int segleft = kSegG - 1;
        bool active = w.rem[0] + w.rem[1] + w.rem[2] > 0;
        while (active) {
          global_pass<DISTINCT>(a, touch_p, col_base(a.d, sc[0], sc[1]) + (sc[2] << 4), 1, n_dpass);
          n_pass++;
          bool mx, my, mz;
          bool out = walk_step(w, mx, my, mz);
          out = out | (mz & (segleft == 0));
          segleft -= mz;
          sc[0] = mod_pos(sc[0] + (mx ? w.sg[0] : 0), nx);
          sc[1] = mod_pos(sc[1] + (my ? w.sg[1] : 0), ny);
          sc[2] = mod_pos(sc[2] + (mz ? w.sg[2] : 0), nz);
          active = !out && (w.rem[0] + w.rem[1] + w.rem[2] > 0);
        }
        continue;
      }
      // binned segment: start from the item's region offsets
      const int doff = item.w & 15, coff = (item.w >> 4) & 63;
      int zs = (item.w >> 10) & 127;
      const int32_t sd = rd0 + doff;
      const int32_t scs = mod_pos(rc0 + coff, nc);
      const int32_t ldv = mod_pos(sd - rod, nd), lcv = mod_pos(scs - roc, nc);
      const int32_t l[3] = {d == 0 ? ldv : lcv, d == 0 ? lcv : ldv, mod_pos(zs - a.d.ro[2], nz)};
      const int32_t v[3] = {a.O[0] + l[0], a.O[1] + l[1], a.O[2] + l[2]};
      Walk w;
      walk_init(a, q, v, l, w);
      const int32_t lz0 = l[2];
      const int32_t sgd = d == 0 ? w.sg[0] : w.sg[1];
      int segleft = sgd > 0 ? min(rd0 + kBinT, nd) - 1 - sd : doff;
      int xo = d == 0 ? doff : coff, yo = d == 0 ? coff : doff;
      int zsteps = 0;
      bool active = w.rem[0] + w.rem[1] + w.rem[2] > 0;
      while (active) {
        const int co = d == 0 ? yo : xo;
        if ((unsigned)co < (unsigned)kBinRows) {
          const int idx = zs * kLevelHalves + (((xo >> 2) * nbyr + (yo >> 2)) << 4) +
                          (((yo & 3) << 2) | (xo & 3));
          atomicAdd(&cnt[idx >> 1], 1u << ((idx & 1) << 4));
        } else {
          const int32_t sx = mod_pos(rx0 + xo, nx), sy = mod_pos(ry0 + yo, ny);
          global_pass<DISTINCT>(a, touch_p, col_base(a.d, sx, sy) + (zs << 4), 1, n_dpass);
        }
        n_pass++;
        bool mx, my, mz;
        bool out = walk_step(w, mx, my, mz);
        const bool md = d == 0 ? mx : my;
        out = out | (md & (segleft == 0));
        segleft -= md;
        xo += mx ? w.sg[0] : 0;
        yo += my ? w.sg[1] : 0;
        zs += mz ? w.sg[2] : 0;
        zs = zs == nz ? 0 : (zs < 0 ? nz - 1 : zs);
        zsteps += mz;
        active = !out && (w.rem[0] + w.rem[1] + w.rem[2] > 0);
      }
      // storage levels of the visited local z range (monotone path)
      const int32_t zlo = w.sg[2] < 0 ? lz0 - zsteps : lz0;
      mark_levels(lev0, lev1, mod_pos(zlo + a.d.ro[2], nz), zsteps + 1, nz);
    }
    if (lev0) atomicOr(&s_lev[0], lev0);
    if (lev1) atomicOr(&s_lev[1], lev1);
    __syncthreads();
    if (glob) continue;
    // ---- flush the touched levels: counters -> passes, counters cleared
    if (tid == 0) {
      int nl = 0;
      for (int k = 0; k < 2; k++) {
        unsigned long long m = s_lev[k];
        while (m) {
          const int b = __ffsll((long long)m) - 1;
          m &= m - 1;
          s_levlist[nl++] = 64 * k + b;
        }
      }
      s_nlev = nl;
      s_lev[0] = 0;
      s_lev[1] = 0;
    }
    __syncthreads();
    const int total = s_nlev * kLevelWords;
    for (int i = tid; i < total; i += kTraceBinThreads) {
      const int li = i / kLevelWords;
      const int wi = i - li * kLevelWords;
      const int z = s_levlist[li];
      const uint32_t val = cnt[z * kLevelWords + wi];
      if (!val) continue;
      cnt[z * kLevelWords + wi] = 0;
#pragma unroll
      for (int hf = 0; hf < 2; hf++) {
        const int32_t cv = (val >> (16 * hf)) & 0xFFFF;
        if (!cv) continue;
        const int idx = 2 * wi + hf;
        const int brick = idx >> 4, inb = idx & 15;
        const int bxo = brick / nbyr, byo = brick - bxo * nbyr;
        const int32_t sx = mod_pos(rx0 + bxo * 4 + (inb & 3), nx);
        const int32_t sy = mod_pos(ry0 + byo * 4 + (inb >> 2), ny);
        global_pass<DISTINCT>(a, touch_p, col_base(a.d, sx, sy) + (z << 4), cv, n_dpass);
      }
    }
  }
  // per-block counters, summed by the host
  const int c3 = wave_sum(n_pass);
  const int c4 = DISTINCT ? wave_sum(n_dpass) : 0;
  if (lane == 0) {
    wsum[wv][0] = c3;
    wsum[wv][1] = c4;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long p = 0, r = 0;
    for (int w = 0; w < kTraceBinThreads / 64; w++) {
      p += wsum[w][0];
      r += wsum[w][1];
    }
    a.part_trace[2 * blockIdx.x] = p;
    a.part_trace[2 * blockIdx.x + 1] = r;
  }
}

// ---------------------------------------------------------------------------
// Batched stages: persistent grids walk the virtual blocks of all maps of a
// batch; block b of a stage belongs to the map m with pre[m] <= b < pre[m+1].
__device__ __forceinline__ int find_map(const int32_t* pre, int n, int vb) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= vb) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_b_clear(const BatchTables* __restrict__ t,
                                                    unsigned long long* stamps,
                                                    unsigned int* done) {
  const int n = t->st.nmaps;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (gid == 0) stamps[0] = wall_clock64();
  constexpr int kWords = 8 + kStripes;
  for (int64_t i = gid; i < (int64_t)n * kWords; i += stride) t->ins[i / kWords].stats[i % kWords] = 0;
  for (int64_t i = gid; i < n; i += stride) done[i] = 0;
  for (int m = 0; m < n; m++) clear_body(t->clr[m], gid, stride);
}

__global__ __launch_bounds__(kRayBlock) void k_b_rays(const BatchTables* __restrict__ t) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_rays[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map(t->st.pre_rays, n, vb);
    rays_body<false>(t->ins[m], vb - t->st.pre_rays[m]);
  }
}

__global__ __launch_bounds__(kBlock) void k_b_trace(const BatchTables* __restrict__ t) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_trace[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map(t->st.pre_trace, n, vb);
    trace_body<false>(t->ins[m], vb - t->st.pre_trace[m], t->ins[m].trace_blocks);
    __syncthreads();
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

hipError_t launch_clear(const ClearArgs& a, hipStream_t s) {
  int64_t total = 0;
  for (int k = 0; k < a.nbox; k++) {
    const int64_t t = (int64_t)a.box[k][1] * a.box[k][3] * a.box[k][5];
    total = t > total ? t : total;
  }
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear, dim3(grid_for(total)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_batch_insert(const BatchTables* tab, const BatchGrid& g,
                               unsigned long long* stamps, unsigned int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_b_clear, dim3(g.clear), dim3(kBlock), 0, s, tab, stamps, done);
  hipLaunchKernelGGL(k_b_rays, dim3(g.rays), dim3(kRayBlock), 0, s, tab);
  hipLaunchKernelGGL(k_b_trace, dim3(g.trace), dim3(kBlock), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

int64_t max_segments_binned(const Dims& d) {
  const int32_t m = d.nx > d.ny ? d.nx : d.ny;
  const int64_t a = m / kBinT + 3, b = (d.nz - 1) / kSegG + 1;
  return a > b ? a : b;
}

size_t rays_bin_lds(int nb) { return (size_t)nb * 4; }

size_t trace_bin_lds(int nz) { return (size_t)kLevelWords * nz * 4; }

int64_t max_segments(const Dims& d, int32_t seg_len) {
  int32_t m = d.nx > d.ny ? d.nx : d.ny;
  if (d.nz > m) m = d.nz;
  return (m - 1) / seg_len + 1;
}

hipError_t launch_rays(const InsertArgs& a, bool distinct, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int g = (a.n + kRayBlock - 1) / kRayBlock;
  if (a.binned) {
    const size_t lds = rays_bin_lds(a.nb);
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)k_rays_bin<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_rays_bin<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    if (distinct)
      hipLaunchKernelGGL(k_rays_bin<true>, dim3(g), dim3(kRayBlock), lds, s, a);
    else
      hipLaunchKernelGGL(k_rays_bin<false>, dim3(g), dim3(kRayBlock), lds, s, a);
    return hipGetLastError();
  }
  if (distinct)
    hipLaunchKernelGGL(k_rays<true>, dim3(g), dim3(kRayBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_rays<false>, dim3(g), dim3(kRayBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_trace(const InsertArgs& a, bool distinct, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (a.binned) {
    hipLaunchKernelGGL(k_binscan, dim3(1), dim3(1024), 0, s, a);
    const size_t lds = trace_bin_lds(a.d.nz);
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void*)k_trace_bin<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_trace_bin<false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    if (distinct)
      hipLaunchKernelGGL(k_trace_bin<true>, dim3(a.tb_blocks), dim3(kTraceBinThreads), lds, s, a);
    else
      hipLaunchKernelGGL(k_trace_bin<false>, dim3(a.tb_blocks), dim3(kTraceBinThreads), lds, s, a);
    return hipGetLastError();
  }
  if (distinct)
    hipLaunchKernelGGL(k_trace<true>, dim3(a.trace_blocks), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_trace<false>, dim3(a.trace_blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace gvom
