// The map buffer of Sec. III-B of arXiv 2109.13176 and the first step of its
// map processing (Sec. III-D): per-scan voxel maps are kept in a buffer and
// combined into one map with one thread per voxel of the combined map.
//
// A buffered map is one scan's map in the storage of Sec. III-A: a lookup
// table with one int32 per voxel (an occupied voxel's index in the data array,
// else -1 - misses), a data array {hits, passes, lowest return} of the
// occupied voxels, and the window origin.  The lookup table is kept in the
// maps' toroidal bricked storage order (world voxel g at storage coordinate
// g mod n per axis), so one world voxel sits at the same index in every
// buffered map whose window holds it and in the combined map: the combine is
// an element-wise pass whose only per-map work is a window test.  The data
// array is in storage order of the occupied voxels.
//
// A scan is turned into its map by the insert path of an internal producer
// map (empty before every push), whose state is then moved into the buffer
// slot and cleared in the same pass.
#include <hip/hip_runtime.h>

#include <new>
#include <utility>
#include <vector>

#include "gvom_internal.h"
#include "map_state.h"

namespace gvom {

namespace {

constexpr int kBrickThreads = 256;  // one block per 4 x 4 brick of columns
constexpr int kMaxDepth = 64;       // buffered maps per combine
static_assert(kBrickThreads == 256, "a block of the count covers 16 bricks of 16 columns");

struct SlotArgs {
  Dims d;
  int32_t* hits;                  // producer state, left empty
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;        // read, then cleared (each block owns its brick's columns)
  int32_t* lut;                   // slot: lookup table in storage order
  map_voxel_t* data;              // slot: data array
  int64_t cap;
  const int32_t* brick_cnt;       // occupied voxels per brick
  const int32_t* group_base;      // exclusive prefix per group of 16 bricks
};

struct CombineArgs {
  Dims d;                         // of the combined map, ring offsets of its new origin
  int32_t O[3];                   // origin of the combined map (the newest buffered map's)
  int32_t k;                      // buffered maps
  const int32_t* lut[kMaxDepth];
  const map_voxel_t* data[kMaxDepth];
  int64_t cap[kMaxDepth];         // data entries written (a slot holds at most one
                                  // occupied voxel per point, so always >= its count)
  int32_t org[kMaxDepth][3];
  int32_t* hits;
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;
};

__device__ __forceinline__ void brick_xy(const Dims& d, int b, int& bx, int& by) {
  bx = b / d.nby;
  by = b - bx * d.nby;
}

// Occupied voxels per brick (one lane per storage column, 16 lanes per brick)
// and per group of 16 bricks (one block).
__global__ __launch_bounds__(kBrickThreads) void k_slot_count(Dims d,
                                                              const unsigned long long* occ,
                                                              int32_t* brick_cnt,
                                                              int32_t* group_cnt, int nbricks) {
  __shared__ int32_t wsum[kBrickThreads / 64];
  const int64_t t = (int64_t)blockIdx.x * kBrickThreads + threadIdx.x;
  const int b = (int)(t >> 4), j = (int)(t & 15);
  int c = 0;
  if (b < nbricks) {
    int bx, by;
    brick_xy(d, b, bx, by);
    const int sx = 4 * bx + (j & 3), sy = 4 * by + (j >> 2);
    if (sx < d.nx && sy < d.ny) {
      const int64_t col = ((int64_t)sx * d.ny + sy) * d.W;
      c = __popcll(occ[col]);
      if (d.W > 1) c += __popcll(occ[col + 1]);
    }
  }
#pragma unroll
  for (int o = 8; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  if (b < nbricks && j == 0) brick_cnt[b] = c;
  int g = j == 0 ? c : 0;
  g += __shfl_xor(g, 16);
  g += __shfl_xor(g, 32);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
#pragma unroll
    for (int w = 0; w < kBrickThreads / 64; w++) sum += wsum[w];
    group_cnt[blockIdx.x] = sum;
  }
}

// Moves the producer's state into the slot, brick by brick in storage order:
// item (level z, quarter q) holds the four storage voxels of columns
// 4q .. 4q+3 of the brick at z, so items are in storage order and the rank of
// an occupied voxel is the brick's base plus a block scan of the item counts.
// Every non-zero passes word is zeroed; hits and lowest return only where
// occupied (they are empty elsewhere); the brick's occupancy words are
// cleared once read.
__global__ __launch_bounds__(kBrickThreads) void k_slot_write(SlotArgs a) {
  __shared__ unsigned long long mlo[16], mhi[16];
  __shared__ int32_t wtot[kBrickThreads / 64];
  __shared__ int32_t sbase;
  const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  int bx, by;
  brick_xy(a.d, b, bx, by);
  if (t < 64) {
    // rank base: the group's prefix plus the bricks of the group before b
    const int first = b & ~15;
    int c = t < 16 && first + t < b ? a.brick_cnt[first + t] : 0;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) c += __shfl_xor(c, o);
    if (t == 0) sbase = a.group_base[b >> 4] + c;
  }
  if (t < 16) {
    const int sx = 4 * bx + (t & 3), sy = 4 * by + (t >> 2);
    unsigned long long lo = 0ull, hi = 0ull;
    if (sx < a.d.nx && sy < a.d.ny) {
      const int64_t col = ((int64_t)sx * a.d.ny + sy) * a.d.W;
      lo = a.occ[col];
      a.occ[col] = 0ull;
      if (a.d.W > 1) {
        hi = a.occ[col + 1];
        a.occ[col + 1] = 0ull;
      }
    }
    mlo[t] = lo;
    mhi[t] = hi;
  }
  __syncthreads();
  const int nz = a.d.nz;
  const int items = nz * 4;
  const int64_t s_b = (int64_t)b * nz * 16;
  int32_t run = sbase;
  for (int i0 = 0; i0 < items; i0 += kBrickThreads) {
    const int i = i0 + t;
    const int z = i >> 2, q = i & 3;
    unsigned bits = 0u;
    if (i < items) {
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int j = 4 * q + e;
        const unsigned long long m = z < 64 ? mlo[j] >> z : mhi[j] >> (z - 64);
        bits |= (unsigned)(m & 1ull) << e;
      }
    }
    // the item's words are read before the rank scan, so their latency
    // overlaps it: passes always, hits and lowest returns (one 16-byte load
    // each) where a voxel of the item is occupied
    const int64_t s = s_b + 16 * z + 4 * q;
    int4 p = make_int4(0, 0, 0, 0), h4, m4;
    if (i < items) p = *(const int4*)(a.passes + s);
    if (bits) {
      h4 = *(const int4*)(a.hits + s);
      m4 = *(const int4*)(a.minqz + s);
    }
    const int c = __popc(bits);
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kBrickThreads / 64; k++) {
      const int v = wtot[k];
      before += k < w ? v : 0;
      total += v;
    }
    int32_t rank = run + before + incl - c;
    run += total;
    if (i < items) {
      const int32_t pv[4] = {p.x, p.y, p.z, p.w};
      int32_t v[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        if ((bits >> e) & 1u) {
          if (rank < a.cap) {
            const int32_t hv[4] = {h4.x, h4.y, h4.z, h4.w};
            const int32_t mv[4] = {m4.x, m4.y, m4.z, m4.w};
            map_voxel_t dv;
            dv.hits = hv[e];
            dv.passes = pv[e];
            dv.min_qz = mv[e];
            a.data[rank] = dv;
          }
          a.hits[s + e] = 0;
          a.minqz[s + e] = INT32_MAX;
          v[e] = rank++;
        } else {
          v[e] = -1 - pv[e];
        }
      }
      *(int4*)(a.lut + s) = make_int4(v[0], v[1], v[2], v[3]);
      // only the few voxels rays passed need clearing
      if (p.x | p.y | p.z | p.w) *(int4*)(a.passes + s) = make_int4(0, 0, 0, 0);
    }
    __syncthreads();  // wtot is rewritten by the next round
  }
}

__device__ __forceinline__ int32_t ring_to_local(int32_t s, int32_t ro, int32_t n) {
  const int32_t l = s - ro;
  return l < 0 ? l + n : l;
}

// Full combination of the voxels of one item selected by `mask`: sums over
// every buffered map whose window holds the voxel (all four voxels of an item
// share y and z, so the map's window test on those is done once).
__device__ __forceinline__ void sum_maps(const CombineArgs& a, const int64_t s,
                                         const int32_t gx[4], const int32_t gy,
                                         const int32_t gz, const unsigned mask, int32_t h[4],
                                         int32_t p[4], int32_t mq[4]) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if ((mask >> e) & 1u) {
      h[e] = 0;
      p[e] = 0;
      mq[e] = INT32_MAX;
    }
  }
  for (int k = 0; k < a.k; k++) {
    if ((uint32_t)(gy - a.org[k][1]) >= (uint32_t)ny ||
        (uint32_t)(gz - a.org[k][2]) >= (uint32_t)nz)
      continue;
    bool in[4], any = false;
#pragma unroll
    for (int e = 0; e < 4; e++) {
      in[e] = ((mask >> e) & 1u) && (uint32_t)(gx[e] - a.org[k][0]) < (uint32_t)nx;
      any |= in[e];
    }
    if (!any) continue;
    const int4 v4 = *(const int4*)(a.lut[k] + s);
    const int32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (!in[e]) continue;
      if (v[e] >= 0) {
        if (v[e] >= a.cap[k]) continue;
        const map_voxel_t dv = a.data[k][v[e]];
        h[e] += dv.hits;
        p[e] += dv.passes;
        mq[e] = min(mq[e], dv.min_qz);
      } else {
        p[e] += -1 - v[e];
      }
    }
  }
}

// The same with the tables of kSumBatch maps read at once (for the full
// combine, where every item reads every map; the in-place update's rare full
// recombinations keep the lean one-map-at-a-time form above).
__device__ __forceinline__ void sum_maps_batched(const CombineArgs& a, const int64_t s,
                                         const int32_t gx[4], const int32_t gy,
                                         const int32_t gz, const unsigned mask, int32_t h[4],
                                         int32_t p[4], int32_t mq[4]) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if ((mask >> e) & 1u) {
      h[e] = 0;
      p[e] = 0;
      mq[e] = INT32_MAX;
    }
  }
  // the tables of kSumBatch maps are read at once (every map's table holds
  // index s, so the loads need no window test; clamped to the last map),
  // then each map's entries are taken where its window holds the voxel
  constexpr int kSumBatch = 8;
  for (int k0 = 0; k0 < a.k; k0 += kSumBatch) {
    int4 vb[kSumBatch];
#pragma unroll
    for (int j = 0; j < kSumBatch; j++) vb[j] = *(const int4*)(a.lut[min(k0 + j, a.k - 1)] + s);
#pragma unroll
    for (int j = 0; j < kSumBatch; j++) {
      const int k = k0 + j;
      if (k >= a.k) break;
      if ((uint32_t)(gy - a.org[k][1]) >= (uint32_t)ny ||
          (uint32_t)(gz - a.org[k][2]) >= (uint32_t)nz)
        continue;
      bool in[4];
#pragma unroll
      for (int e = 0; e < 4; e++)
        in[e] = ((mask >> e) & 1u) && (uint32_t)(gx[e] - a.org[k][0]) < (uint32_t)nx;
      const int32_t v[4] = {vb[j].x, vb[j].y, vb[j].z, vb[j].w};
#pragma unroll
      for (int e = 0; e < 4; e++) {
        if (!in[e]) continue;
        if (v[e] >= 0) {
          if (v[e] >= a.cap[k]) continue;
          const map_voxel_t dv = a.data[k][v[e]];
          h[e] += dv.hits;
          p[e] += dv.passes;
          mq[e] = min(mq[e], dv.min_qz);
        } else {
          p[e] += -1 - v[e];
        }
      }
    }
  }
}

// World coordinates of an item's voxels in the combined window.
__device__ __forceinline__ unsigned item_world(const CombineArgs& a, const int bx, const int by,
                                               const int z, const int q, int32_t gx[4],
                                               int32_t& gy, int32_t& gz) {
  const int sy = 4 * by + q;
  gy = a.O[1] + ring_to_local(sy, a.d.ro[1], a.d.ny);
  gz = a.O[2] + ring_to_local(z, a.d.ro[2], a.d.nz);
  unsigned valid = 0u;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    const int sx = 4 * bx + e;
    if (sx < a.d.nx && sy < a.d.ny) valid |= 1u << e;
    gx[e] = a.O[0] + ring_to_local(sx, a.d.ro[0], a.d.nx);
  }
  return valid;
}

__device__ __forceinline__ void set_occ(unsigned long long* mlo, unsigned long long* mhi,
                                        const int j, const int z, const bool on) {
  unsigned long long* w = z < 64 ? &mlo[j] : &mhi[j];
  const unsigned long long bit = 1ull << (z & 63);
  if (on) atomicOr(w, bit);
  else atomicAnd(w, ~bit);
}

// The combined map's state, brick by brick: each item's four voxels are
// located in world coordinates, looked up at the same storage index in every
// buffered map whose window holds them, and summed; the occupancy words of
// the brick's columns are assembled in LDS.
__global__ __launch_bounds__(kBrickThreads) void k_combine(const CombineArgs a) {
  __shared__ unsigned long long mlo[16], mhi[16];
  const int b = blockIdx.x, t = threadIdx.x;
  if (t < 16) mlo[t] = mhi[t] = 0ull;
  __syncthreads();
  int bx, by;
  brick_xy(a.d, b, bx, by);
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int items = nz * 4;
  const int64_t s_b = (int64_t)b * nz * 16;
  for (int i = t; i < items; i += kBrickThreads) {
    const int z = i >> 2, q = i & 3;
    const int64_t s = s_b + 16 * z + 4 * q;
    int32_t gx[4], gy, gz;
    const unsigned valid = item_world(a, bx, by, z, q, gx, gy, gz);
    int32_t h[4] = {0, 0, 0, 0}, p[4] = {0, 0, 0, 0};
    int32_t mq[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    sum_maps_batched(a, s, gx, gy, gz, valid, h, p, mq);
    *(int4*)(a.hits + s) = make_int4(h[0], h[1], h[2], h[3]);
    *(int4*)(a.passes + s) = make_int4(p[0], p[1], p[2], p[3]);
    *(int4*)(a.minqz + s) = make_int4(mq[0], mq[1], mq[2], mq[3]);
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (h[e] > 0) set_occ(mlo, mhi, 4 * q + e, z, true);
  }
  __syncthreads();
  if (t < 16) {
    const int sx = 4 * bx + (t & 3), sy = 4 * by + (t >> 2);
    if (sx < nx && sy < ny) {
      const int64_t col = ((int64_t)sx * ny + sy) * a.d.W;
      a.occ[col] = mlo[t];
      if (a.d.W > 1) a.occ[col + 1] = mhi[t];
    }
  }
}

// Update of a combined map that holds the combination of the buffer as it
// was one push ago: the buffer has since gained its newest map and lost at
// most one map (evicted).  Hits and misses are sums, so a voxel of the old
// window changes by the newest map's counts minus the evicted map's; voxels
// where neither map has anything are not touched.  A minimum cannot be taken
// back: where the evicted map's lowest return equals the combined minimum,
// and for every voxel that entered with the new window, the voxel is
// combined in full.  Same result as k_combine.
struct IncArgs {
  int32_t O_old[3];               // origin of the combination being updated
  const int32_t* nw_lut;          // newest map (its window is the combined window)
  const map_voxel_t* nw_data;
  int64_t nw_cap;
  int32_t has_ev;                 // a map was evicted by the newest push
  const int32_t* ev_lut;
  const map_voxel_t* ev_data;
  int64_t ev_cap;
  int32_t ev_org[3];
};

// One item of the update (all lanes of a wave call it together: the evicted
// minima are recombined wave-wide).  n4 / e4_all: the item's entries in the
// newest and the evicted map's tables.
__device__ __forceinline__ void inc_item(const CombineArgs& a, const IncArgs& u, const int i,
                                         const bool active, const int lane,
                                         const int32_t* my_lut, const map_voxel_t* my_data,
                                         const int64_t my_cap, const int32_t* my_org,
                                         const int4 n4, const int4 e4_all) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int per_brick = nz * 4;
  const int ic = active ? i : 0;
  const int b = ic / per_brick;
  const int r = ic - b * per_brick;
  const int z = r >> 2, q = r & 3;
  int bx, by;
  brick_xy(a.d, b, bx, by);
  const int64_t s = (int64_t)ic << 2;
  int32_t gx[4], gy, gz;
  const unsigned valid = item_world(a, bx, by, z, q, gx, gy, gz) & (active ? 15u : 0u);
  const bool old_yz = (uint32_t)(gy - u.O_old[1]) < (uint32_t)ny &&
                      (uint32_t)(gz - u.O_old[2]) < (uint32_t)nz;
  const bool ev_yz = u.has_ev && (uint32_t)(gy - u.ev_org[1]) < (uint32_t)ny &&
                     (uint32_t)(gz - u.ev_org[2]) < (uint32_t)nz;
  const int4 e4 = ev_yz ? e4_all : make_int4(-1, -1, -1, -1);
  const int32_t nw[4] = {n4.x, n4.y, n4.z, n4.w};
  int32_t ev[4] = {e4.x, e4.y, e4.z, e4.w};
  unsigned enter = 0u, upd = 0u, hit = 0u, evo = 0u;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if ((uint32_t)(gx[e] - u.ev_org[0]) >= (uint32_t)nx) ev[e] = -1;
    if (!((valid >> e) & 1u)) continue;
    const bool in_old = old_yz && (uint32_t)(gx[e] - u.O_old[0]) < (uint32_t)nx;
    if (!in_old) enter |= 1u << e;
    else if (ev[e] >= 0) evo |= 1u << e;
    else if (ev[e] != -1 || nw[e] != -1) upd |= 1u << e;
    if (nw[e] >= 0) hit |= 1u << e;
  }
  // only misses change where neither map has a return: hits and lowest
  // return are read and written where a map has one or the voxel is
  // combined in full
  const unsigned hm = enter | evo | (upd & hit);
  int32_t h[4] = {0, 0, 0, 0}, p[4] = {0, 0, 0, 0}, mq[4] = {0, 0, 0, 0};
  if (enter | evo | upd) {
    const int4 p4 = *(const int4*)(a.passes + s);
    p[0] = p4.x; p[1] = p4.y; p[2] = p4.z; p[3] = p4.w;
  }
  if (hm) {
    const int4 h4 = *(const int4*)(a.hits + s);
    const int4 m4 = *(const int4*)(a.minqz + s);
    h[0] = h4.x; h[1] = h4.y; h[2] = h4.z; h[3] = h4.w;
    mq[0] = m4.x; mq[1] = m4.y; mq[2] = m4.z; mq[3] = m4.w;
  }
  const int32_t h_old[4] = {h[0], h[1], h[2], h[3]};
  map_voxel_t evd[4];
  unsigned coop = 0u;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if (!((evo >> e) & 1u)) continue;
    // the evicted map's lowest return is above the combined minimum: the
    // minimum stays, its counts come off; otherwise the voxel is combined
    // again from every map
    if (ev[e] < u.ev_cap) evd[e] = u.ev_data[ev[e]];
    if (ev[e] < u.ev_cap && evd[e].min_qz > mq[e]) upd |= 1u << e;
    else coop |= 1u << e;
  }
  // voxels that entered with the window: dense (whole slabs), each lane
  // combines its own
  if (enter) sum_maps(a, s, gx, gy, gz, enter, h, p, mq);
  // voxels whose minimum went with the evicted map: scattered, so the wave
  // combines them one at a time with one lane per buffered map
  unsigned long long lanes = __ballot(coop != 0u);
  while (lanes) {
    const int L = __ffsll((long long)lanes) - 1;
    lanes &= lanes - 1;
    const unsigned cm = (unsigned)__builtin_amdgcn_readlane((int)coop, L);
    const int iL = __builtin_amdgcn_readlane(ic, L);
    const int gyL = __builtin_amdgcn_readlane(gy, L);
    const int gzL = __builtin_amdgcn_readlane(gz, L);
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (!((cm >> e) & 1u)) continue;
      const int gxL = __builtin_amdgcn_readlane(gx[e], L);
      int32_t hh = 0, pp = 0, mm = INT32_MAX;
      if (lane < a.k && (uint32_t)(gxL - my_org[0]) < (uint32_t)nx &&
          (uint32_t)(gyL - my_org[1]) < (uint32_t)ny &&
          (uint32_t)(gzL - my_org[2]) < (uint32_t)nz) {
        const int32_t v = my_lut[((int64_t)iL << 2) + e];
        if (v >= 0) {
          if (v < my_cap) {
            const map_voxel_t dv = my_data[v];
            hh = dv.hits;
            pp = dv.passes;
            mm = dv.min_qz;
          }
        } else {
          pp = -1 - v;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        hh += __shfl_xor(hh, o);
        pp += __shfl_xor(pp, o);
        mm = min(mm, __shfl_xor(mm, o));
      }
      if (lane == L) {
        h[e] = hh;
        p[e] = pp;
        mq[e] = mm;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if (!((upd >> e) & 1u)) continue;
    if (ev[e] >= 0) {
      h[e] -= evd[e].hits;
      p[e] -= evd[e].passes;
    } else if (ev[e] < -1) {
      p[e] -= -1 - ev[e];
    }
    if (nw[e] >= 0) {
      if (nw[e] < u.nw_cap) {
        const map_voxel_t dv = u.nw_data[nw[e]];
        h[e] += dv.hits;
        p[e] += dv.passes;
        mq[e] = min(mq[e], dv.min_qz);
      }
    } else {
      p[e] += -1 - nw[e];
    }
  }
  if (enter | evo | upd) *(int4*)(a.passes + s) = make_int4(p[0], p[1], p[2], p[3]);
  if (hm) {
    *(int4*)(a.hits + s) = make_int4(h[0], h[1], h[2], h[3]);
    *(int4*)(a.minqz + s) = make_int4(mq[0], mq[1], mq[2], mq[3]);
    // occupancy bit = hits >= 1; flip it only where that changed (the old
    // bit of an entering voxel belongs to the voxel that left)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (!((hm >> e) & 1u) || (h_old[e] > 0) == (h[e] > 0)) continue;
      unsigned long long* w =
          a.occ + ((int64_t)(4 * bx + e) * ny + (4 * by + q)) * a.d.W + (z >> 6);
      const unsigned long long bit = 1ull << (z & 63);
      if (h[e] > 0) atomicOr(w, bit);
      else atomicAnd(w, ~bit);
    }
  }
}

// Classification of an item for the update: does any voxel change (entered
// the window, or the newest or the evicted map has something there)?
__device__ __forceinline__ bool inc_changed(const CombineArgs& a, const IncArgs& u, const int i,
                                            const int4 n4, const int4 e4_all) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int per_brick = nz * 4;
  const int b = i / per_brick;
  const int r = i - b * per_brick;
  const int z = r >> 2, q = r & 3;
  int bx, by;
  brick_xy(a.d, b, bx, by);
  int32_t gx[4], gy, gz;
  const unsigned valid = item_world(a, bx, by, z, q, gx, gy, gz);
  const bool old_yz = (uint32_t)(gy - u.O_old[1]) < (uint32_t)ny &&
                      (uint32_t)(gz - u.O_old[2]) < (uint32_t)nz;
  const bool ev_yz = u.has_ev && (uint32_t)(gy - u.ev_org[1]) < (uint32_t)ny &&
                     (uint32_t)(gz - u.ev_org[2]) < (uint32_t)nz;
  const int32_t nw[4] = {n4.x, n4.y, n4.z, n4.w};
  const int32_t ev4[4] = {e4_all.x, e4_all.y, e4_all.z, e4_all.w};
  bool changed = false;
#pragma unroll
  for (int e = 0; e < 4; e++) {
    if (!((valid >> e) & 1u)) continue;
    const int32_t ev = ev_yz && (uint32_t)(gx[e] - u.ev_org[0]) < (uint32_t)nx ? ev4[e] : -1;
    const bool in_old = old_yz && (uint32_t)(gx[e] - u.O_old[0]) < (uint32_t)nx;
    changed |= !in_old || ev != -1 || nw[e] != -1;
  }
  return changed;
}

// Pass 1 of the update: stream both tables once and list the items that
// change, per block (block b's list holds the items of its grid-stride walk,
// at most `cap`).
__global__ __launch_bounds__(kBrickThreads) void k_inc_find(const CombineArgs a, const IncArgs u,
                                                            int32_t* __restrict__ list,
                                                            int32_t* __restrict__ cnt,
                                                            const int cap) {
  __shared__ int32_t scount;
  if (threadIdx.x == 0) scount = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int n_items = (int)(a.d.vs >> 2);
  const int stride = gridDim.x * kBrickThreads;
  int32_t* mine = list + (int64_t)blockIdx.x * cap;
  for (int base = blockIdx.x * kBrickThreads; base < n_items; base += stride) {
    const int i = base + threadIdx.x;
    bool changed = false;
    if (i < n_items) {
      const int4 n4 = *(const int4*)(u.nw_lut + ((int64_t)i << 2));
      const int4 e4 = u.has_ev ? *(const int4*)(u.ev_lut + ((int64_t)i << 2))
                               : make_int4(-1, -1, -1, -1);
      changed = inc_changed(a, u, i, n4, e4);
    }
    const unsigned long long m = __ballot(changed);
    int wbase = 0;
    if (lane == 0 && m) wbase = atomicAdd(&scount, __popcll(m));
    wbase = __shfl(wbase, 0);
    if (changed) mine[wbase + __popcll(m & ((1ull << lane) - 1ull))] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = scount;
}

// Pass 2: every listed item updated (the list order does not matter: items
// are disjoint, and occupancy bits are flipped by atomics).
__global__ __launch_bounds__(kBrickThreads) void k_combine_inc(const CombineArgs a,
                                                               const IncArgs u,
                                                               const int32_t* __restrict__ list,
                                                               const int32_t* __restrict__ cnt,
                                                               const int cap) {
  const int lane = threadIdx.x & 63;
  // lane j holds buffered map j for the wave-wide recombination
  const int32_t* my_lut = nullptr;
  const map_voxel_t* my_data = nullptr;
  int64_t my_cap = 0;
  int32_t my_org[3] = {0, 0, 0};
  for (int k = 0; k < a.k; k++) {
    if (lane == k) {
      my_lut = a.lut[k];
      my_data = a.data[k];
      my_cap = a.cap[k];
      my_org[0] = a.org[k][0];
      my_org[1] = a.org[k][1];
      my_org[2] = a.org[k][2];
    }
  }
  const int c = cnt[blockIdx.x];
  const int32_t* mine = list + (int64_t)blockIdx.x * cap;
  // the bound is uniform per block, so every lane reaches the wave-wide step
  for (int j0 = 0; j0 < c; j0 += kBrickThreads) {
    const int j = j0 + threadIdx.x;
    const bool active = j < c;
    const int i = active ? mine[j] : 0;
    int4 n4 = make_int4(-1, -1, -1, -1), e4 = make_int4(-1, -1, -1, -1);
    if (active) {
      n4 = *(const int4*)(u.nw_lut + ((int64_t)i << 2));
      if (u.has_ev) e4 = *(const int4*)(u.ev_lut + ((int64_t)i << 2));
    }
    inc_item(a, u, i, active, lane, my_lut, my_data, my_cap, my_org, n4, e4);
  }
}

int64_t n_bricks(const Dims& d) { return (int64_t)((d.nx + 3) / 4) * d.nby; }

}  // namespace

}  // namespace gvom

struct map_buffer_t {
  map_params_t p;
  int32_t depth;                // buffered maps
  int32_t ring;                 // slots = depth + 1: the map the last push evicted
                                // stays readable until the next push
  hipStream_t stream;           // producer stream: pushes run here
  map_t* prod;                  // producer map, empty between pushes
  struct Slot {
    int32_t* lut;
    map_voxel_t* data;
    int64_t cap;
    int32_t origin[3];
  };
  std::vector<Slot> slots;      // push j lives in slot j mod ring
  int64_t npush;                // pushes since create / reset
  int32_t* brick_cnt;           // per brick: occupied voxels
  int32_t* group_cnt;           // per 16 bricks: occupied voxels, then their prefix
  int64_t* n_occ;               // [ring] occupied voxels per slot (device)
  hipEvent_t pushed;            // recorded after every push
  // combines that may still read the slots: the latest event per output
  // stream (work on one stream completes in order)
  std::vector<std::pair<hipStream_t, hipEvent_t>> pending;
  std::vector<hipEvent_t> pool;
  // the last combine: a combine into the same, unchanged map one push later
  // updates it instead of combining every buffered map again
  bool incremental;
  int32_t* inc_list;            // the update's per-block lists of changed items
  int32_t* inc_cnt;             // [inc_grid] listed items per block
  int inc_grid, inc_cap;        // blocks of the update passes; list slots per block
  map_t* last_out;
  uint64_t last_version;
  int64_t last_npush;
  int32_t sticky;
};

namespace {

int32_t buf_fail(map_buffer_t* b, hipError_t e) {
  if (e == hipSuccess) return MAP_OK;
  (void)hipGetLastError();
  b->sticky = MAP_E_DEVICE;
  return MAP_E_DEVICE;
}

// Orders the producer stream after every combine that may still read a slot.
hipError_t wait_combines(map_buffer_t* b) {
  hipError_t e = hipSuccess;
  for (const auto& pe : b->pending) {
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, pe.second, 0);
    b->pool.push_back(pe.second);
  }
  b->pending.clear();
  return e;
}

int32_t held(const map_buffer_t* b) {
  return (int32_t)(b->npush < b->depth ? b->npush : b->depth);
}

map_buffer_t::Slot& slot_of(map_buffer_t* b, int64_t push) { return b->slots[push % b->ring]; }

}  // namespace

extern "C" {

int32_t map_buffer_create(const map_params_t* p, int32_t depth, void* stream,
                          map_buffer_t** out) {
  if (!out) return MAP_E_INVALID;
  *out = nullptr;
  if (depth < 1 || depth > gvom::kMaxDepth) return MAP_E_INVALID;
  map_t* prod = nullptr;
  int32_t st = map_create(p, stream, &prod);
  if (st) return st;
  map_buffer_t* b = new (std::nothrow) map_buffer_t();
  if (!b) {
    map_destroy(prod);
    return MAP_E_OOM;
  }
  b->p = *p;
  b->depth = depth;
  b->ring = depth + 1;
  b->stream = (hipStream_t)stream;
  b->prod = prod;
  b->slots.assign(b->ring, map_buffer_t::Slot{nullptr, nullptr, 0, {0, 0, 0}});
  b->npush = 0;
  b->incremental = true;
  {
    const int64_t items = prod->d.vs / 4;
    int64_t grid = (items + gvom::kBrickThreads - 1) / gvom::kBrickThreads;
    if (grid > (int64_t)prod->n_cu * 8) grid = (int64_t)prod->n_cu * 8;
    const int64_t rounds = (items + grid * gvom::kBrickThreads - 1) / (grid * gvom::kBrickThreads);
    b->inc_grid = (int)grid;
    b->inc_cap = (int)(rounds * gvom::kBrickThreads);
  }
  b->last_out = nullptr;
  b->sticky = MAP_OK;
  const int64_t nb = gvom::n_bricks(prod->d);
  hipError_t e = gvom::dev_alloc((void**)&b->brick_cnt, (size_t)nb * 4);
  if (e == hipSuccess) e = gvom::dev_alloc((void**)&b->group_cnt, (size_t)((nb + 15) / 16) * 4);
  if (e == hipSuccess) e = gvom::dev_alloc((void**)&b->n_occ, (size_t)b->ring * 8);
  if (e == hipSuccess)
    e = gvom::dev_alloc((void**)&b->inc_list, (size_t)b->inc_grid * b->inc_cap * 4);
  if (e == hipSuccess) e = gvom::dev_alloc((void**)&b->inc_cnt, (size_t)b->inc_grid * 4);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->pushed, hipEventDisableTiming);
  else b->pushed = nullptr;
  for (int i = 0; i < b->ring && e == hipSuccess; i++) {
    e = gvom::dev_alloc((void**)&b->slots[i].lut, (size_t)prod->d.vs * 4);
    if (e != hipSuccess) b->slots[i].lut = nullptr;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    map_buffer_destroy(b);
    return MAP_E_OOM;
  }
  *out = b;
  return MAP_OK;
}

int32_t map_buffer_destroy(map_buffer_t* b) {
  if (!b) return MAP_OK;
  (void)hipStreamSynchronize(b->stream);
  for (const auto& pe : b->pending) {
    (void)hipEventSynchronize(pe.second);
    (void)hipEventDestroy(pe.second);
  }
  for (hipEvent_t ev : b->pool) (void)hipEventDestroy(ev);
  for (auto& s : b->slots) {
    (void)gvom::dev_free(s.lut);
    (void)gvom::dev_free(s.data);
  }
  (void)gvom::dev_free(b->brick_cnt);
  (void)gvom::dev_free(b->group_cnt);
  (void)gvom::dev_free(b->n_occ);
  (void)gvom::dev_free(b->inc_list);
  (void)gvom::dev_free(b->inc_cnt);
  if (b->pushed) (void)hipEventDestroy(b->pushed);
  map_destroy(b->prod);
  (void)hipGetLastError();
  delete b;
  return MAP_OK;
}

int32_t map_buffer_reset(map_buffer_t* b) {
  if (!b) return MAP_E_INVALID;
  (void)hipStreamSynchronize(b->stream);
  for (const auto& pe : b->pending) {
    (void)hipEventSynchronize(pe.second);
    b->pool.push_back(pe.second);
  }
  b->pending.clear();
  (void)hipGetLastError();
  b->npush = 0;
  b->last_out = nullptr;
  b->sticky = MAP_OK;
  return map_reset(b->prod);
}

int32_t map_buffer_set_incremental(map_buffer_t* b, int32_t enable) {
  if (!b) return MAP_E_INVALID;
  b->incremental = enable != 0;
  return MAP_OK;
}

int32_t map_buffer_push(map_buffer_t* b, const float* xyz_dev, int64_t n, const float pose[12],
                        uint32_t flags) {
  if (!b) return MAP_E_INVALID;
  if (b->sticky) return b->sticky;
  map_t* m = b->prod;
  // a scan that is not recentred takes the newest buffered window
  int32_t o[3];
  if (b->npush > 0) {
    const map_buffer_t::Slot& nw = slot_of(b, b->npush - 1);
    o[0] = nw.origin[0];
    o[1] = nw.origin[1];
    o[2] = nw.origin[2];
  } else {
    o[0] = -m->p.nx / 2;
    o[1] = -m->p.ny / 2;
    o[2] = -m->p.sensor_z_voxel;
  }
  gvom::set_empty_origin(m, o);
  hipError_t e = wait_combines(b);
  if (e != hipSuccess) return buf_fail(b, e);
  // a fresh window holds at most one occupied voxel per point
  const int32_t si = (int32_t)(b->npush % b->ring);
  map_buffer_t::Slot& s = b->slots[si];
  const int64_t need = n < m->d.vs ? (n > 0 ? n : 1) : m->d.vs;
  if (need > s.cap) {
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return buf_fail(b, e);
    const int64_t want = s.cap > 0 && need < 2 * s.cap ? 2 * s.cap : need;
    (void)gvom::dev_free(s.data);
    s.data = nullptr;
    s.cap = 0;
    if (gvom::dev_alloc((void**)&s.data, (size_t)want * sizeof(map_voxel_t)) != hipSuccess) {
      (void)hipGetLastError();
      s.data = nullptr;
      return MAP_E_OOM;
    }
    s.cap = want;
  }
  int32_t st = map_insert_scan(m, xyz_dev, n, pose, flags);
  if (st) {
    if (m->sticky) b->sticky = m->sticky;
    return st;
  }
  const gvom::Dims& d = m->d;
  const int64_t nb = gvom::n_bricks(d);
  const int ng = (int)((nb + 15) / 16);  // one block of the count per 16 bricks
  hipLaunchKernelGGL(gvom::k_slot_count, dim3((unsigned)ng), dim3(gvom::kBrickThreads), 0,
                     b->stream, d, m->occ, b->brick_cnt, b->group_cnt, (int)nb);
  e = hipGetLastError();
  if (e == hipSuccess) e = gvom::launch_scan_i32(b->group_cnt, ng, b->n_occ + si, b->stream);
  if (e == hipSuccess) {
    gvom::SlotArgs a;
    a.d = d;
    a.hits = m->hits;
    a.passes = m->passes;
    a.minqz = m->minqz;
    a.occ = m->occ;
    a.lut = s.lut;
    a.data = s.data;
    a.cap = s.cap;
    a.brick_cnt = b->brick_cnt;
    a.group_base = b->group_cnt;
    hipLaunchKernelGGL(gvom::k_slot_write, dim3((unsigned)nb), dim3(gvom::kBrickThreads), 0,
                       b->stream, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(b->pushed, b->stream);
  if (e != hipSuccess) {
    m->sticky = MAP_E_DEVICE;
    return buf_fail(b, e);
  }
  m->empty = true;
  m->lut_counted = false;
  m->version = gvom::next_version();
  s.origin[0] = m->origin[0];
  s.origin[1] = m->origin[1];
  s.origin[2] = m->origin[2];
  b->npush++;
  return MAP_OK;
}

int32_t map_buffer_combine(map_buffer_t* b, map_t* out) {
  if (!b || !out) return MAP_E_INVALID;
  if (b->sticky) return b->sticky;
  if (out->sticky) return out->sticky;
  if (out->p.nx != b->p.nx || out->p.ny != b->p.ny || out->p.nz != b->p.nz ||
      out->p.res_m != b->p.res_m)
    return MAP_E_INVALID;
  if (b->npush == 0) return MAP_E_INVALID;
  hipEvent_t ev = nullptr;
  if (!b->pool.empty()) {
    ev = b->pool.back();
    b->pool.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return MAP_E_DEVICE;
  }
  // `out` still holds this buffer's combination of one push ago
  const bool inc = b->incremental && b->last_out == out && out->version == b->last_version &&
                   b->npush == b->last_npush + 1;
  gvom::IncArgs u;
  if (inc) {
    for (int i = 0; i < 3; i++) u.O_old[i] = out->origin[i];
    const map_buffer_t::Slot& nw = slot_of(b, b->npush - 1);
    u.nw_lut = nw.lut;
    u.nw_data = nw.data;
    u.nw_cap = nw.cap;
    const int64_t evicted = b->npush - 1 - b->depth;  // push that left the buffer
    u.has_ev = evicted >= 0;
    const map_buffer_t::Slot& es = slot_of(b, evicted >= 0 ? evicted : 0);
    u.ev_lut = es.lut;
    u.ev_data = es.data;
    u.ev_cap = es.cap;
    for (int i = 0; i < 3; i++) u.ev_org[i] = es.origin[i];
  }
  hipError_t e = hipStreamWaitEvent(out->stream, b->pushed, 0);
  const map_buffer_t::Slot& nw = slot_of(b, b->npush - 1);
  gvom::set_origin(out, nw.origin);
  out->lut_counted = false;
  out->empty = false;
  gvom::CombineArgs a;
  a.d = out->d;
  for (int i = 0; i < 3; i++) a.O[i] = nw.origin[i];
  a.k = held(b);
  for (int j = 0; j < a.k; j++) {
    const map_buffer_t::Slot& s = slot_of(b, b->npush - a.k + j);
    a.lut[j] = s.lut;
    a.data[j] = s.data;
    a.cap[j] = s.cap;
    for (int i = 0; i < 3; i++) a.org[j][i] = s.origin[i];
  }
  a.hits = out->hits;
  a.passes = out->passes;
  a.minqz = out->minqz;
  a.occ = out->occ;
  if (e == hipSuccess) {
    const dim3 blk(gvom::kBrickThreads);
    if (inc) {
      // list the changed items while streaming both tables, then update them
      const dim3 g((unsigned)b->inc_grid);
      hipLaunchKernelGGL(gvom::k_inc_find, g, blk, 0, out->stream, a, u, b->inc_list, b->inc_cnt,
                         b->inc_cap);
      hipLaunchKernelGGL(gvom::k_combine_inc, g, blk, 0, out->stream, a, u, b->inc_list,
                         b->inc_cnt, b->inc_cap);
    } else {
      hipLaunchKernelGGL(gvom::k_combine, dim3((unsigned)gvom::n_bricks(out->d)), blk, 0,
                         out->stream, a);
    }
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev, out->stream);
  out->version = gvom::next_version();
  if (e != hipSuccess) {
    b->pool.push_back(ev);
    (void)hipGetLastError();
    out->sticky = MAP_E_DEVICE;
    b->last_out = nullptr;
    return MAP_E_DEVICE;
  }
  bool replaced = false;
  for (auto& pe : b->pending) {
    if (pe.first == out->stream) {
      b->pool.push_back(pe.second);  // implied by the new event on the same stream
      pe.second = ev;
      replaced = true;
    }
  }
  if (!replaced) b->pending.emplace_back(out->stream, ev);
  b->last_out = out;
  b->last_version = out->version;
  b->last_npush = b->npush;
  return MAP_OK;
}

int32_t map_buffer_count(const map_buffer_t* b) { return b ? held(b) : MAP_E_INVALID; }

int32_t map_buffer_get_stats(map_buffer_t* b, map_stats_t* out) {
  if (!b) return MAP_E_INVALID;
  return map_get_stats(b->prod, out);
}

}  // extern "C"
