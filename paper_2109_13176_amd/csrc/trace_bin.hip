// Binned ray traversal (optional mode of the ray pass, Sec. III-C of
// arXiv 2109.13176): rays cut at storage slabs, passes counted per slab tile
// in LDS and added to the map in storage order.  Results are identical to
// the segmented traversal in insert.hip.
#include "ray_common.h"

namespace gvom {

namespace {

// Storage columns are cut into slabs of kBinT cells along x and along y.  A
// ray whose dominant axis d is x or y is cut where its storage coordinate
// along d enters a new slab, so every piece (segment) lies in one slab.  A
// segment is binned by d, the direction of its cross axis c, its slab g and
// the kBinT-tile h of its start's storage c coordinate.  The bin's region is
// the slab x kBinRows storage rows along c from the tile towards the side the
// ray moves to x all z levels; it holds every voxel of the segment except, at
// most, a few of a short steep ray, which go to global memory directly.
// Persistent work groups take the units (up to kUnit segments of one bin)
// round-robin; a group counts the unit's passes in 16-bit LDS counters laid out like
// the storage bricks, then adds the counters of the touched z levels to the
// passes array with coalesced atomics (regions of different units overlap).
// Rays whose dominant axis is z go to the last bin; they are cut every kSegG
// cells from the sensor and traced with global atomics.

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
__global__ __launch_bounds__(kRayBinBlock) void k_rays_bin(InsertArgs a) {
  extern __shared__ int hist[];  // a.nb counters, then exclusive offsets
  __shared__ unsigned int wcount[kRayBinBlock / 64][4];
  __shared__ int wtot[kRayBinBlock / 64];
  __shared__ long long s_base;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  const int blk = blockIdx.x;
  for (int i = threadIdx.x; i < a.nb; i += kRayBinBlock) hist[i] = 0;
  int32_t q[3];
  PointFlags pf;
  const bool ray = point_pass<DISTINCT>(a, blk * kRayBinBlock + threadIdx.x, q, pf);
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
  const int per = (a.nb + kRayBinBlock - 1) / kRayBinBlock;
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
    for (int w = 0; w < kRayBinBlock / 64; w++) {
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
    a.bin_ent[(int64_t)bin * a.maxblk + blk] = make_int2((int)(base + off), cnt);
    if (cnt) atomicAdd(&a.bin_tot[bin], cnt);
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
// long ones start early) and the bin counters cleared for the next scan.
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
    a.bin_tot[bin] = 0;
  }
  if (threadIdx.x == 0) a.uctl[0] = F + P;
}

// Adds one pass to storage voxel e (global memory), with its distinct bit.
template <bool DISTINCT>
__device__ __forceinline__ void global_pass(const InsertArgs& a, uint32_t* touch_p, int32_t e,
                                            int32_t cnt, int& n_dpass, int& n_upd) {
  atomicAdd(&a.passes[e], cnt);
  n_upd++;
  if (DISTINCT) {
    const uint32_t bit = 1u << (e & 31);
    const uint32_t old = atomicOr(&touch_p[(uint32_t)e >> 5], bit);
    n_dpass += !(old & bit);
  }
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
  __shared__ int wsum[kTraceBinThreads / 64][3];
  const int tid = threadIdx.x, lane = __lane_id(), wv = tid >> 6;
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int32_t dims[3] = {nx, ny, nz};
  for (int i = tid; i < kLevelWords * nz; i += kTraceBinThreads) cnt[i] = 0;
  if (tid == 0) {
    s_lev[0] = 0;
    s_lev[1] = 0;
  }
  uint32_t* touch_p = DISTINCT ? a.touch + ((a.d.vs + 31) >> 5) : nullptr;
  int n_pass = 0, n_dpass = 0, n_upd = 0;
  const int n_units = a.uctl[0];
  // units are dealt round-robin (a shared work counter costs more than the
  // imbalance: same-address atomics serialise in memory)
  for (int u = blockIdx.x; u < n_units; u += gridDim.x) {
    __syncthreads();
    if (tid == 0) s_unit = a.units[u];
    __syncthreads();
    const int4 un = s_unit;
    const int bin = un.x;
    const int nent = a.maxblk;
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
          global_pass<DISTINCT>(a, touch_p, col_base(a.d, sc[0], sc[1]) + (sc[2] << 4), 1, n_dpass, n_upd);
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
          global_pass<DISTINCT>(a, touch_p, col_base(a.d, sx, sy) + (zs << 4), 1, n_dpass, n_upd);
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
        global_pass<DISTINCT>(a, touch_p, col_base(a.d, sx, sy) + (z << 4), cv, n_dpass, n_upd);
      }
    }
  }
  // per-block counters, summed by the host
  const int c3 = wave_sum(n_pass);
  const int c4 = DISTINCT ? wave_sum(n_dpass) : 0;
  const int c6 = wave_sum(n_upd);
  if (lane == 0) {
    wsum[wv][0] = c3;
    wsum[wv][1] = c4;
    wsum[wv][2] = c6;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long p = 0, r = 0, u = 0;
    for (int w = 0; w < kTraceBinThreads / 64; w++) {
      p += wsum[w][0];
      r += wsum[w][1];
      u += wsum[w][2];
    }
    a.part_trace[4 * blockIdx.x] = p;
    a.part_trace[4 * blockIdx.x + 1] = r;
    a.part_trace[4 * blockIdx.x + 2] = u;
    a.part_trace[4 * blockIdx.x + 3] = 0;
  }
}

}  // namespace

int64_t max_segments_binned(const Dims& d) {
  const int32_t m = d.nx > d.ny ? d.nx : d.ny;
  const int64_t a = m / kBinT + 3, b = (d.nz - 1) / kSegG + 1;
  return a > b ? a : b;
}

size_t rays_bin_lds(int nb) { return (size_t)nb * 4; }

size_t trace_bin_lds(int nz) { return (size_t)kLevelWords * nz * 4; }

hipError_t launch_rays_bin(const InsertArgs& a, bool distinct, hipStream_t s) {
  const int gb = (a.n + kRayBinBlock - 1) / kRayBinBlock;
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
    hipLaunchKernelGGL(k_rays_bin<true>, dim3(gb), dim3(kRayBinBlock), lds, s, a);
  else
    hipLaunchKernelGGL(k_rays_bin<false>, dim3(gb), dim3(kRayBinBlock), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_trace_bin(const InsertArgs& a, bool distinct, hipStream_t s) {
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

}  // namespace gvom
