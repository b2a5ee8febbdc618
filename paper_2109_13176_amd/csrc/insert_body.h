// Device bodies of the scan-insertion kernels (Sec. III-C of arXiv 2109.13176):
// the ray pass, the traversal with its line tables and sensor box, the
// sensor-box fold and the window-scroll clears.  Each body does the work of
// one (virtual) block, so the single-map kernels and the batched persistent
// kernel share them.
#pragma once
#include <math.h>

#include "ray_common.h"

namespace gvom {

namespace {


// ---------------------------------------------------------------------------
// Pass 1, one lane per point: transform, record the return in its voxel, and
// cut the ray into segments for the traversal pass.
//
// A ray's voxel path is monotone in every axis.  Along its dominant axis (the
// axis with the most voxel steps) the path is cut every seg_len voxels:
// segment j holds the path voxels whose dominant coordinate lies j*seg_len ..
// (j+1)*seg_len - 1 voxels from the sensor's.  Only segments that start
// inside the window along the dominant axis count.
//
// The block then regroups its rays by segment count (most first; rays of
// equal count keep their order, so neighbouring rays stay together) and
// writes their records {Q, segments} in that order: a traversal wave holds
// segment j of 64 rays that all have it, instead of 64 neighbouring rays of
// which the short ones ended long before j.  Each group of 64 records with at
// most s segments publishes s wave items {group, j}.
constexpr int kRayWaves = kRayBlock / 64;
constexpr int kSegBins = 64;  // segment counts >= kSegBins - 1 share a bin
static_assert(kSegBins * kRayWaves == kRayBlock, "one scan entry per thread");

// Exclusive prefix sum over the block (one value per thread); wtot is
// kRayWaves words of the caller's LDS.
__device__ __forceinline__ int block_excl_scan(int v, int* wtot) {
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wtot[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int w = 0; w < kRayWaves; w++) {
      const int c = wtot[w];
      wtot[w] = s;
      s += c;
    }
  }
  __syncthreads();
  return x - v + wtot[wv];
}

template <bool DISTINCT>
__device__ __forceinline__ void rays_body(const InsertArgs& a, const int blk) {
  __shared__ unsigned int wcount[kRayWaves][5];
  __shared__ unsigned long long wbase[kRayWaves];
  __shared__ int bin_pre[kSegBins * kRayWaves];  // [bin][wave]: count, then prefix
  __shared__ int wtot[kRayWaves];
  __shared__ int4 srec[kRayBlock];
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int i = blk * kRayBlock + threadIdx.x;
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  int32_t q[3];
  PointFlags pf;
  const bool ray = point_pass<DISTINCT>(a, i, q, pf);
  const HitReads hr = record_hit_issue(a, pf);  // completed after the block's returning atomic
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
      const int32_t Sd = sel3(dom, a.S[0], a.S[1], a.S[2]);
      const int32_t lc = (Sd >> 16) - sel3(dom, a.O[0], a.O[1], a.O[2]);
      const int32_t room = sel3(dom, q[0], q[1], q[2]) > Sd ? sel3(dom, dims[0], dims[1], dims[2]) - 1 - lc : lc;
      nseg = min(sel3(dom, n[0], n[1], n[2]), room) / a.seg_len + 1;
    }
  }

  // ---- stable counting sort of the block's rays by bin (most segments first)
  const int bin = kSegBins - 1 - min(nseg, kSegBins - 1);
  unsigned long long peers = ~0ull;  // lanes of this wave in the same bin
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const bool bit = (bin >> k) & 1;
    const unsigned long long m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  const int rank = __popcll(peers & ((1ull << lane) - 1ull));
  bin_pre[threadIdx.x] = 0;
  __syncthreads();
  if (rank == 0) bin_pre[bin * kRayWaves + wv] = __popcll(peers);
  __syncthreads();
  const int pre = block_excl_scan(bin_pre[threadIdx.x], wtot);
  bin_pre[threadIdx.x] = pre;  // every thread read its entry before the scan's barriers
  __syncthreads();
  srec[bin_pre[bin * kRayWaves + wv] + rank] = make_int4(q[0], q[1], q[2], nseg);
  __syncthreads();
  const int4 rec = srec[threadIdx.x];
  a.rays[i] = rec;

  // ---- reserve the wave items: one returning atomic per block, group bases
  // from the block's prefix
  int maxseg = rec.w;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) maxseg = max(maxseg, __shfl_xor(maxseg, o));
  const int c0 = __popcll(__ballot(nonfinite));
  const int c1 = __popcll(__ballot(outrange));
  const int c2 = __popcll(__ballot(hit));
  const int c5 = DISTINCT ? __popcll(__ballot(dhit)) : 0;
  if (lane == 0) {
    wcount[wv][0] = maxseg;
    wcount[wv][1] = c0;
    wcount[wv][2] = c1;
    wcount[wv][3] = c2;
    wcount[wv][4] = c5;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum = 0, s0 = 0, s1 = 0, s2 = 0, s5 = 0;
    for (int w = 0; w < kRayWaves; w++) {
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
    for (int w = 0; w < kRayWaves; w++) wbase[w] += b + a.stripe_off[st];
    unsigned long long* pr = a.part_rays + 4 * (size_t)blk;
    pr[0] = s0;
    pr[1] = s1;
    pr[2] = s2;
    pr[3] = s5;
  }
  __syncthreads();
  record_hit_finish(a, pf, hr, q[2]);
  const int gw = blk * kRayWaves + wv;  // this group's rays: 64 gw .. 64 gw + 63
  const unsigned long long off = wbase[wv];
  for (int j = lane; j < maxseg; j += 64) a.witems[off + j] = make_int2(gw, j);
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
// pairwise differences E_ab = num_a |D_b| - num_b |D_a|, which change by
// constant increments when an axis steps (kept as 32-bit high parts, see
// Walk).  When several axes share the smallest time, the axes moving up step
// first (the shared boundary belongs to the upper cell) and the axes moving
// down step in the next iteration, so the voxel at that instant is visited.
//
// Counting.  Device atomics are charged per (instruction, 64-byte line) at
// the memory side, and the 64 rays of a wave item pass a compact set of lines
// (about 15 on the 64-beam workload, against about 60 line requests when
// every step adds its voxels straight to the map).  So each wave counts its
// item in a private LDS line table: kWtSlots slots of one 64-byte storage
// line each (16 counters of 16 bits, two per word: a voxel takes at most one
// pass per lane of the item, so a counter stays below 65 while it is in the
// table; and a tag = storage index >> 4), found by a hash of
// the line with kWtProbe linear probes and claimed by compare-and-swap; a lane
// remembers the slot of its current line, so it looks up only when its ray
// enters another line.  When the item is done the wave adds every non-zero
// counter of its claimed slots to the map, 16 lanes per line (one line request
// per line), and empties the table.  A line that finds no slot on its probe
// path is added to the map directly.  With BOX, voxels in the sensor box add
// into the block's LDS copy of the box instead, which the block flushes into
// its replica at the end (k_box_fold adds the replicas into the map).  Every
// pass ends up in exactly one counter that reaches the map once, so the
// result is the same integer sum whatever the claim order.
constexpr int kWtSlots = 64;     // slots per wave (one per lane at the flush)
constexpr int kWtStride = 9;     // LDS words per slot: 8 counter pairs + 1 (bank spread)
constexpr int kWtProbe = 4;
constexpr int32_t kWtEmpty = -1;

struct WaveTable {
  int32_t tag[kWtSlots];
  uint32_t cnt[kWtSlots * kWtStride];
  int32_t lst[kWtSlots];
};

// Orders the LDS accesses of one wave's lanes (a wave's LDS operations are
// executed in issue order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Slot of storage line `line` in the wave's table, claiming an empty one on
// its probe path; -1 when the path holds other lines only.  The first slot
// is a multiplicative (Fibonacci) hash of the line's low 24 bits: the top six
// bits of their product with 2^24 / golden ratio (Knuth, TAOCP vol. 3,
// 6.4), one 24-bit multiply.  Tags hold the whole line, so lines that share
// low bits only share a probe path.
__device__ __forceinline__ int wt_lookup(WaveTable& wt, const int32_t line) {
  const uint32_t h = mad_u24((uint32_t)line & 0xFFFFFFu, 0x9E3779u, 0u);
  const int s0 = (int)(h >> 26);
#pragma unroll
  for (int p = 0; p < kWtProbe; p++) {
    const int s = (s0 + p) & (kWtSlots - 1);
    int32_t t = wt.tag[s];
    if (t == kWtEmpty) t = atomicCAS(&wt.tag[s], kWtEmpty, line);
    if (t == kWtEmpty || t == line) return s;
  }
  return -1;
}

// box_cnt[kBoxCells] and wtab[NT / 64] are the block's LDS (the caller's).
template <bool DISTINCT, bool BOX, int NT>
__device__ __forceinline__ void trace_body(const InsertArgs& a, const int blk, const int nblk,
                                           int32_t* box_cnt, WaveTable* wtab) {
  const int lane = __lane_id();
  WaveTable& wt = wtab[threadIdx.x >> 6];
  wt.tag[lane] = kWtEmpty;
  for (int i = lane; i < kWtSlots * kWtStride; i += 64) wt.cnt[i] = 0;
  if (BOX) {
    for (int i = threadIdx.x; i < kBoxCells; i += NT) box_cnt[i] = 0;
  }
  __syncthreads();
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int32_t dims[3] = {nx, ny, nz};
  // wave items of stripe t occupy [stripe_off[t], stripe_off[t] + cnt[t]); the
  // loop runs over their concatenation.  The stripe prefix lives in LDS
  // (in registers it would cost the kernel its last wave per SIMD).
  __shared__ int64_t s_pre[kStripes + 1];
  __shared__ int64_t s_base[kStripes];  // stripe_off[t] - s_pre[t]
  if (threadIdx.x == 0) {
    int64_t p = 0;
#pragma unroll
    for (int t = 0; t < kStripes; t++) {
      s_pre[t] = p;
      s_base[t] = a.stripe_off[t] - p;
      p += min((int64_t)a.stats[8 + t], a.stripe_cap[t]);
    }
    s_pre[kStripes] = p;
  }
  __syncthreads();
  const int64_t count = s_pre[kStripes];  // wave items
  const int64_t stride = (int64_t)nblk * (NT / 64);
  uint32_t* touch_p = DISTINCT ? a.touch + ((a.d.vs + 31) >> 5) : nullptr;
  int32_t* const passes = a.passes;  // kept in registers across the loop
  int n_pass = 0, n_dpass = 0, n_upd = 0;  // n_pass is wave-uniform

  for (int64_t u = (int64_t)blk * (NT / 64) + (threadIdx.x >> 6); u < count; u += stride) {
    bool active = false, near = false;
    Walk w = {};
    int32_t cnt[3] = {0, 0, 0};
    bool stop[3] = {false, false, false};
    int32_t sc[3] = {0, 0, 0};
    int32_t sidx = 0;
    {
      // last stripe t with s_pre[t] <= u (empty stripes share their prefix)
      int t = 0;
#pragma unroll
      for (int step = kStripes / 2; step >= 1; step >>= 1)
        if (u >= s_pre[t + step]) t += step;
      const int2 item = a.witems[s_base[t] + u];
      const int4 ray = a.rays[(int64_t)item.x * 64 + lane];
      const int32_t q[3] = {ray.x, ray.y, ray.z};
      const int j = item.y;
      int32_t sv[3], n[3], sg[3], ad[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        sv[k] = a.S[k] >> 16;
        const int32_t ev = q[k] >> 16;
        n[k] = ev > sv[k] ? ev - sv[k] : sv[k] - ev;
        const int32_t dq = q[k] - a.S[k];
        sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
        ad[k] = dq < 0 ? -dq : dq;
      }
      const int dom = dominant_axis(n);
      int32_t v[3] = {sv[0], sv[1], sv[2]};
      bool inside = j < ray.w;  // the ray has segment j
      const int32_t sgd = sel3(dom, sg[0], sg[1], sg[2]);
      if (inside && j > 0)
        entry_voxel(a.S, sg, ad, dom, sel3(dom, sv[0], sv[1], sv[2]) + sgd * j * a.seg_len, v);
      int32_t l[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        l[k] = v[k] - a.O[k];
        inside = inside && l[k] >= 0 && l[k] < dims[k];
      }
      if (inside) {
        walk_init(a, q, v, l, w);
        budget_init(w, dom, a.seg_len, cnt, stop);
#pragma unroll
        for (int k = 0; k < 3; k++) sc[k] = wrap_add(l[k] + a.d.ro[k], dims[k]);
        sidx = col_base24(a.d, sc[0], sc[1]) + (sc[2] << 4);
        active = (cnt[0] | cnt[1] | cnt[2]) != 0;
        if (BOX) {
          // the segment's dominant-axis cells (window-local) against the box's
          const int32_t c0 = sel3(dom, l[0], l[1], l[2]), c1 = c0 + sgd * (a.seg_len - 1);
          const int32_t lo = c0 < c1 ? c0 : c1, hi = c0 < c1 ? c1 : c0;
          const int32_t bl = sel3(dom, a.box_l[0], a.box_l[1], a.box_l[2]);
          near = hi >= bl && lo < bl + sel3(dom, a.box_e[0], a.box_e[1], a.box_e[2]);
        }
      }
    }
    // box lookups only in waves that can reach the box
    const bool wnear = BOX && __any(near);

    // per-lane constants of the storage wrap
    const bool px = w.sg[0] > 0, py = w.sg[1] > 0, pz = w.sg[2] > 0;
    const int32_t trig0 = px ? nx : -1, trig1 = py ? ny : -1, trig2 = pz ? nz : -1;
    const int32_t wv0 = px ? 0 : nx - 1, wv1 = py ? 0 : ny - 1, wv2 = pz ? 0 : nz - 1;
    int32_t cur_line = kWtEmpty;  // this lane's current line and its slot
    int cur_slot = -1;
    for (;;) {
      const unsigned long long ab = __ballot(active);
      if (!ab) break;
      n_pass += __popcll(ab);
      // ---- one pass of the current voxel
      if (active) {
        int bidx = -1;
        if (BOX && wnear) {
          // storage offsets from the box's first cell (unsigned: wrapped)
          const uint32_t d0 = (uint32_t)wrap_add(sc[0] - a.box_s[0] + nx, nx);
          const uint32_t d1 = (uint32_t)wrap_add(sc[1] - a.box_s[1] + ny, ny);
          const uint32_t d2 = (uint32_t)wrap_add(sc[2] - a.box_s[2] + nz, nz);
          if (d0 < (uint32_t)a.box_e[0] && d1 < (uint32_t)a.box_e[1] && d2 < (uint32_t)a.box_e[2])
            bidx = (int)((d0 * kBoxXY + d1) * kBoxZ + d2);
        }
        if (BOX && bidx >= 0) {
          atomicAdd(&box_cnt[bidx], 1);
        } else {
          const int32_t line = sidx >> 4;
          if (line != cur_line) {
            cur_line = line;
            cur_slot = wt_lookup(wt, line);
          }
          if (cur_slot >= 0) {
            atomicAdd(&wt.cnt[cur_slot * kWtStride + ((sidx & 15) >> 1)], 1u << ((sidx & 1) << 4));
          } else {
            n_upd++;
            atomicAdd(&passes[sidx], 1);
            if (DISTINCT) {
              const uint32_t bit = 1u << (sidx & 31);
              const uint32_t old = atomicOr(&touch_p[(uint32_t)sidx >> 5], bit);
              n_dpass += !(old & bit);
            }
          }
        }
      }
      // ---- step
      bool mx, my, mz;
      const bool out = budget_step(w, cnt, stop, px, py, pz, mx, my, mz);
      const int32_t t0 = sc[0] + (mx ? w.sg[0] : 0);
      const int32_t t1 = sc[1] + (my ? w.sg[1] : 0);
      const int32_t t2 = sc[2] + (mz ? w.sg[2] : 0);
      sc[0] = t0 == trig0 ? wv0 : t0;
      sc[1] = t1 == trig1 ? wv1 : t1;
      sc[2] = t2 == trig2 ? wv2 : t2;
      sidx = col_base24(a.d, sc[0], sc[1]) + (sc[2] << 4);
      active = active & !out & ((cnt[0] | cnt[1] | cnt[2]) != 0);
    }
    // ---- flush the wave's table: 16 lanes per claimed line
    wave_lds_sync();
    const int32_t tg = wt.tag[lane];
    const unsigned long long vm = __ballot(tg != kWtEmpty);
    if (vm) {
      if (tg != kWtEmpty) wt.lst[__popcll(vm & ((1ull << lane) - 1ull))] = lane;
      wave_lds_sync();
      const int nv = __popcll(vm);
      const int w = lane & 15;
      for (int k = 0; k < nv; k += 4) {
        const int e = k + (lane >> 4);
        if (e < nv) {
          const int s = wt.lst[e];
          const uint32_t pair = wt.cnt[s * kWtStride + (w >> 1)];
          const int c = (int)((pair >> ((w & 1) << 4)) & 0xFFFFu);
          // both lanes of a pair have read it before the even one clears it
          if (pair && !(w & 1)) wt.cnt[s * kWtStride + (w >> 1)] = 0;
          if (c) {
            const int32_t addr = (wt.tag[s] << 4) + w;
            n_upd++;
            atomicAdd(&passes[addr], c);
            if (DISTINCT) {
              const uint32_t bit = 1u << (addr & 31);
              const uint32_t old = atomicOr(&touch_p[(uint32_t)addr >> 5], bit);
              n_dpass += !(old & bit);
            }
          }
        }
      }
      wave_lds_sync();
      wt.tag[lane] = kWtEmpty;
      wave_lds_sync();
    }
  }
  if (BOX) {
    // flush the block's box counts into its replica (coalesced; zero cells
    // are skipped)
    __syncthreads();
    int32_t* rep = a.box_rep + (size_t)(blk % kBoxReps) * kBoxCells;
    for (int i = threadIdx.x; i < kBoxCells; i += NT) {
      const int32_t c = box_cnt[i];
      if (c) atomicAdd(&rep[i], c);
    }
  }
  // per-block counters, written without atomics (summed by the host)
  __shared__ int wsum[NT / 64][3];
  const int c3 = n_pass;
  const int c4 = DISTINCT ? wave_sum(n_dpass) : 0;
  const int c6 = wave_sum(n_upd);
  if (lane == 0) {
    wsum[threadIdx.x >> 6][0] = c3;
    wsum[threadIdx.x >> 6][1] = c4;
    wsum[threadIdx.x >> 6][2] = c6;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long p = 0, q = 0, u = 0;
    for (int w = 0; w < NT / 64; w++) {
      p += wsum[w][0];
      q += wsum[w][1];
      u += wsum[w][2];
    }
    a.part_trace[4 * blk] = p;
    a.part_trace[4 * blk + 1] = q;
    a.part_trace[4 * blk + 2] = u;
    a.part_trace[4 * blk + 3] = 0;
  }
}

// Sensor-box fold: thread (cell i, group g) sums cell i over the kFoldReps
// replicas of group g (zeroing them for the next insert) and adds the sum to
// the cell's passes.  Distinct passes of box cells are counted here (the
// traversal skipped them): the group whose bit-or finds the cell's bit clear
// counts it.  Block b (linear over the grid) writes its counters to slot
// trace_blocks + b.
constexpr int kFoldReps = 8;
constexpr int kFoldGroups = kBoxReps / kFoldReps;
static_assert(kBoxReps % kFoldReps == 0, "replica groups");

constexpr int kFoldCellBlocks = (kBoxCells + kBlock - 1) / kBlock;

// Fold block (cell block bx, replica group by) of one map.  Block (0, 0)
// also zeroes the ray pass's segment counters for the next insert (the
// traversal, which read them, has finished).
template <bool DISTINCT>
__device__ __forceinline__ void box_fold_body(const InsertArgs& a, const int bx, const int by) {
  if (bx == 0 && by == 0 && threadIdx.x < kStripes) a.stats[8 + threadIdx.x] = 0ull;
  const int i = bx * kBlock + threadIdx.x;
  int n_dpass = 0;
  if (i < kBoxCells) {
    int32_t v[kFoldReps];
    int32_t* p = a.box_rep + (size_t)by * kFoldReps * kBoxCells + i;
#pragma unroll
    for (int r = 0; r < kFoldReps; r++) v[r] = p[(size_t)r * kBoxCells];
    int32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kFoldReps; r++) {
      sum += v[r];
      if (v[r]) p[(size_t)r * kBoxCells] = 0;
    }
    const int dz = i % kBoxZ, t = i / kBoxZ;
    const int dy = t % kBoxXY, dx = t / kBoxXY;
    if (sum && dx < a.box_e[0] && dy < a.box_e[1] && dz < a.box_e[2]) {
      const int32_t sx = wrap_add(a.box_s[0] + dx, a.d.nx);
      const int32_t sy = wrap_add(a.box_s[1] + dy, a.d.ny);
      const int32_t sz = wrap_add(a.box_s[2] + dz, a.d.nz);
      const int32_t idx = col_base(a.d, sx, sy) + (sz << 4);
      atomicAdd(&a.passes[idx], sum);
      if (DISTINCT) {
        uint32_t* touch_p = a.touch + ((a.d.vs + 31) >> 5);
        const uint32_t bit = 1u << (idx & 31);
        const uint32_t old = atomicOr(&touch_p[(uint32_t)idx >> 5], bit);
        n_dpass = !(old & bit);
      }
    }
  }
  __shared__ int wsum[kBlock / 64];
  const int c = DISTINCT ? wave_sum(n_dpass) : 0;
  if (__lane_id() == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long q = 0;
    for (int w = 0; w < kBlock / 64; w++) q += wsum[w];
    const size_t slot = (size_t)a.trace_blocks + by * kFoldCellBlocks + bx;
    unsigned long long* pt = a.part_trace + 4 * slot;
    pt[0] = 0;
    pt[1] = q;
    pt[2] = 0;
    pt[3] = 0;
  }
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

}  // namespace
}  // namespace gvom
