// Device bodies of the export kernels (Sec. III-A and III-D of arXiv
// 2109.13176): the per-column reduction, the slope / roughness /
// negative-obstacle tiles and the lookup-table passes.  Each body does the
// work of one (virtual) block, so the single-map kernels and the batched
// persistent kernel share them.
#pragma once
#include <math.h>

#include "ray_common.h"

namespace gvom {

namespace {

constexpr uint32_t kQNaN = 0x7FC00000u;


// Column occupancy in window-local z order (bit z = local z), nz <= 128.
struct Mask128 {
  unsigned long long lo, hi;
};

__device__ __forceinline__ Mask128 local_mask(const unsigned long long* occ, int64_t col,
                                              int W, int nz, int roz) {
  unsigned __int128 m = occ[col * W];
  if (W > 1) m |= (unsigned __int128)occ[col * W + 1] << 64;
  if (roz != 0) {
    const unsigned __int128 full =
        nz == 128 ? ~(unsigned __int128)0 : (((unsigned __int128)1 << nz) - 1);
    m = ((m >> roz) | (m << (nz - roz))) & full;
  }
  Mask128 r;
  r.lo = (unsigned long long)m;
  r.hi = (unsigned long long)(m >> 64);
  return r;
}

__device__ __forceinline__ int lowest_bit(const Mask128& m) {
  if (m.lo) return __ffsll((long long)m.lo) - 1;
  if (m.hi) return 64 + __ffsll((long long)m.hi) - 1;
  return -1;
}

__device__ __forceinline__ bool test_bit(const Mask128& m, int z) {
  return z < 64 ? ((m.lo >> z) & 1ull) : ((m.hi >> (z - 64)) & 1ull);
}

// popcount of the bits below z
__device__ __forceinline__ int rank_below(const Mask128& m, int z) {
  if (z < 64) return __popcll(m.lo & ((1ull << z) - 1ull));
  const int zh = z - 64;
  return __popcll(m.lo) + __popcll(m.hi & ((1ull << zh) - 1ull));
}

// Position of the set bit of rank r (0 = lowest) of m; r < popcount(m).
// Halving search: at each width s the bits of the lower s positions are
// counted and the search moves up past them when r is not among them.
__device__ __forceinline__ int select_bit(const Mask128& m, int r) {
  const int pl = __popcll(m.lo);
  unsigned long long w = r < pl ? m.lo : m.hi;
  int pos = r < pl ? 0 : 64;
  r = r < pl ? r : r - pl;
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) {
    const int c = __popcll(w & ((1ull << sh) - 1ull));
    if (r >= c) {
      r -= c;
      w >>= sh;
      pos += sh;
    }
  }
  return pos;
}

// One lane per map column (window-local pixel).  Ground voxel = lowest
// occupied voxel; height = its lowest return.  The positive-obstacle band is
// the occupied voxels n_lo..n_hi above the ground voxel; its density is
// sum(hits) / sum(hits + passes); hard iff that ratio exceeds num/den
// (compared exactly in integers), soft otherwise.
// With a.colpre set it also does the table export's counting pass (the
// occupied voxels of every column, ranked within its group of 64 columns;
// see lut_count_body), from the occupancy mask it loads anyway.
__device__ __forceinline__ void column_counts(const ColumnArgs& a, const int c, const int cnt) {
  const int lane = __lane_id();
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  const int C = a.d.nx * a.d.ny;
  if (c < C) a.colpre[c] = incl - cnt;
  if (lane == 63 && (c >> 6) * 64 < C) a.block_base[c >> 6] = incl;
}

__device__ __forceinline__ void column_body(const ColumnArgs& a, const int blk) {
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz;
  const int c = blk * kBlock + threadIdx.x;
  const bool valid = c < nx * ny;
  int sx = 0, sy = 0;
  Mask128 m = {0ull, 0ull};
  if (valid) {
    const int x = c / ny, y = c - x * ny;
    sx = wrap_add(x + a.d.ro[0], nx);
    sy = wrap_add(y + a.d.ro[1], ny);
    m = local_mask(a.occ, (int64_t)sx * ny + sy, a.d.W, nz, a.d.ro[2]);
  }
  // every lane of the wave takes part in the rank scan
  if (a.colpre) column_counts(a, c, __popcll(m.lo) + __popcll(m.hi));
  if (!valid) return;
  const int kg = lowest_bit(m);
  float height = __uint_as_float(kQNaN), density = __uint_as_float(kQNaN);
  int32_t hq = INT32_MIN;
  uint8_t f = 0;
  if (kg >= 0) {
    const int64_t base = col_base(a.d, sx, sy);
    hq = a.minqz[base + (wrap_add(kg + a.d.ro[2], nz) << 4)];
    height = (float)((double)hq * a.res / 65536.0);
    f = 1;
    int64_t sh = 0, sa = 0;
    int cnt = 0;
    const int zlo = kg + a.n_lo;
    const int zhi = min(kg + a.n_hi, nz - 1);
    // the band's occupied levels in chunks of eight, all loads of a chunk in
    // flight before the sums (one memory round trip per chunk)
    for (int z0 = zlo; z0 <= zhi; z0 += 8) {
      int32_t hv[8], pv[8];
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int z = z0 + u;
        hv[u] = pv[u] = -1;
        if (z <= zhi && test_bit(m, z)) {
          const int64_t e = base + (wrap_add(z + a.d.ro[2], nz) << 4);
          hv[u] = a.hits[e];
          pv[u] = a.passes[e];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; u++) {
        if (hv[u] < 0) continue;
        sh += hv[u];
        sa += (int64_t)hv[u] + pv[u];
        cnt++;
      }
    }
    if (cnt > 0) {
      density = (float)((double)sh / (double)sa);
      const bool hard = sh * a.dens_den > (int64_t)a.dens_num * sa;
      f |= 2 | (hard ? 4 : 8);
    }
  }
  a.height[c] = height;
  a.density[c] = density;
  a.flags[c] = f;
  a.hq[c] = hq;
}


// 2D surface maps on tiles of TILE x TILE pixels (kPix / NT per thread)
// with a halo of H = max(half_fit, D) pixels staged in LDS.  Defined pixels
// get the N x N least-squares plane (integer normal equations, exact
// determinant, Cramer's rule in double); undefined pixels get the four-cone
// negative-obstacle search.
//
// Cone test: ring d of the +x cone of pixel (x, y) is the slice of staged row
// x+d over columns y-d..y+d; it holds a defined cell iff the distance along
// that row from column y to the nearest defined cell is <= d.  These row
// (and column) distances are precomputed for the tile's own columns (rows)
// from per-line bit masks, so each ring costs one LDS byte; only the slice
// where a cone stops is then read cell by cell.
constexpr int kTile = 32;
constexpr int kSurfThreads = kTile * kTile;
constexpr int kMaxMaskWords = 3;  // staged edge <= 192 cells

__device__ __forceinline__ unsigned long long span_bits(unsigned long long v, int w, int a,
                                                        int b) {
  // bits of word w that fall in the inclusive cell range [a, b]
  const int lo = a - 64 * w, hi = b - 64 * w;
  if (lo > 0) v &= ~0ull << lo;
  if (hi < 63) v &= ~0ull >> (63 - hi);
  return v;
}

// distance from cell k of a line (bit mask of MW words, T cells) to its
// nearest set bit, clamped to 255
__device__ __forceinline__ int line_distance(const unsigned long long* L, int MW, int T, int k) {
  int best = 255;
  for (int w = 0; w < MW; w++) {
    unsigned long long v = L[w];
    if (!v) continue;
    // nearest set bit at or below k, and at or above k, within this word
    const int base = 64 * w;
    if (k >= base) {
      const int top = min(k - base, 63);
      const unsigned long long below = top == 63 ? v : (v & ((2ull << top) - 1ull));
      if (below) best = min(best, k - (base + 63 - __clzll((long long)below)));
    }
    if (k <= base + 63) {
      const int bot = max(k - base, 0);
      const unsigned long long above = v & (~0ull << bot);
      if (above) best = min(best, base + __ffsll((long long)above) - 1 - k);
    }
  }
  (void)T;
  return best;
}

// LDS row stride of the staged heights: odd, so that the column reads of
// the mask pass hit distinct banks
__host__ __device__ __forceinline__ int surface_stride(int T) { return T | 1; }

template <int NT, int TILE>
__device__ __forceinline__ void surface_body(const SurfaceArgs& a, const int H, const int bx,
                                             const int by) {
  constexpr int kPix = TILE * TILE;  // tile pixels
  static_assert(kPix % NT == 0 && NT % 64 == 0 && kPix % 64 == 0, "tile pixels per thread");
  extern __shared__ int32_t lds[];
  const int T = TILE + 2 * H;          // staged tile edge
  const int TS = surface_stride(T);     // LDS row stride of th
  const int MW = (T + 63) >> 6;         // mask words per staged row / column
  int32_t* th = lds;                                                    // [T][TS]
  unsigned long long* rmask = (unsigned long long*)(lds + ((T * TS + 1) & ~1));  // [T][MW]
  unsigned long long* cmask = rmask + T * MW;                            // [T][MW]
  uint8_t* rdist = (uint8_t*)(cmask + T * MW);  // [T][TILE]: row r, tile column j
  uint8_t* cdist = rdist + T * TILE;           // [T][TILE]: column c, tile row i
  const int gx0 = bx * TILE - H, gy0 = by * TILE - H;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  constexpr int kWaves = NT / 64;            // waves of the block
  constexpr int kVW = kPix / 64;     // 64-pixel groups of the tile
  constexpr int kPer = kPix / NT;    // tile pixels per thread
  // stage the heights row by row (a wave per row, lanes along y); the
  // ballot of each 64-cell piece is that row's mask word.  A wave issues the
  // loads of kSurfRows rows before it stores any (addresses clamped into the
  // map, so every load is in bounds; cells outside it take the empty value).
  constexpr int kSurfRows = 4;
  for (int r0 = wv; r0 < T; r0 += kSurfRows * kWaves) {
    int32_t v[kSurfRows][kMaxMaskWords];
#pragma unroll
    for (int j = 0; j < kSurfRows; j++) {
      const int64_t rowc = (int64_t)min(max(gx0 + r0 + j * kWaves, 0), a.nx - 1) * a.ny;
#pragma unroll
      for (int w = 0; w < kMaxMaskWords; w++)
        v[j][w] = a.hq[rowc + min(max(gy0 + 64 * w + lane, 0), a.ny - 1)];
    }
#pragma unroll
    for (int j = 0; j < kSurfRows; j++) {
      const int r = r0 + j * kWaves;
      if (r >= T) break;
      const int gx = gx0 + r;
      const bool rowok = gx >= 0 && gx < a.nx;
#pragma unroll
      for (int w = 0; w < kMaxMaskWords; w++) {
        if (w >= MW) break;
        const int k = 64 * w + lane;
        const int gy = gy0 + k;
        const int32_t x = rowok && k < T && gy >= 0 && gy < a.ny ? v[j][w] : INT32_MIN;
        if (k < T) th[r * TS + k] = x;
        const unsigned long long b = __ballot(x != INT32_MIN);
        if (lane == 0) rmask[r * MW + w] = b;
      }
    }
  }
  __syncthreads();
  // column masks: lanes along x
  for (int c = wv; c < T; c += kWaves) {
    for (int w = 0; w < MW; w++) {
      const int k = 64 * w + lane;
      const bool d = k < T && th[k * TS + c] != INT32_MIN;
      const unsigned long long b = __ballot(d);
      if (lane == 0) cmask[c * MW + w] = b;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * T * TILE; i += NT) {
    const bool col = i >= T * TILE;
    const int ii = col ? i - T * TILE : i;
    const int line = ii / TILE, j = ii - line * TILE;
    const int dd = line_distance((col ? cmask : rmask) + line * MW, MW, T, H + j);
    (col ? cdist : rdist)[ii] = (uint8_t)dd;
  }

  // defined pixels (plane fit) and undefined ones (cone search) go to
  // separate waves: the block's pixels are listed defined-first, ranks from
  // ballots (deterministic order)
  __shared__ int16_t order[kPix];
  __shared__ int wcnt[kVW][2];
  bool pdef[kPer], pund[kPer];
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int p = k * NT + (int)threadIdx.x;  // tile pixel; group p >> 6 = k * kWaves + wv
    const int px = p / TILE, py = p - px * TILE;
    const int gx = bx * TILE + px, gy = by * TILE + py;
    const bool valid = gx < a.nx && gy < a.ny;
    pdef[k] = valid && th[(px + H) * TS + py + H] != INT32_MIN;
    pund[k] = valid && !pdef[k];
    const unsigned long long bd = __ballot(pdef[k]), bu = __ballot(pund[k]);
    if (lane == 0) {
      wcnt[p >> 6][0] = __popcll(bd);
      wcnt[p >> 6][1] = __popcll(bu);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const int p = k * NT + (int)threadIdx.x;
    int pd = 0, pu = 0;
    for (int w = 0; w < (p >> 6); w++) {
      pd += wcnt[w][0];
      pu += wcnt[w][1];
    }
    const unsigned long long bd = __ballot(pdef[k]), bu = __ballot(pund[k]);
    const int below_d = __builtin_amdgcn_mbcnt_hi((uint32_t)(bd >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bd, 0));
    const int below_u = __builtin_amdgcn_mbcnt_hi((uint32_t)(bu >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bu, 0));
    if (pdef[k]) order[pd + below_d] = (int16_t)p;
    if (pund[k]) order[kPix - 1 - (pu + below_u)] = (int16_t)p;
  }
  __syncthreads();
  int nd = 0, nu = 0;
  for (int w = 0; w < kVW; w++) {
    nd += wcnt[w][0];
    nu += wcnt[w][1];
  }
  // slots [0, nd): defined pixels, [kPix - nu, kPix): undefined
  for (int slot = threadIdx.x; slot < kPix; slot += NT) {
  if (slot >= nd && slot < kPix - nu) continue;
  const int me = order[slot];
  const int px = me / TILE, py = me - px * TILE;
  const int gx = bx * TILE + px, gy = by * TILE + py;
  const int h = a.half_fit, D = a.search_d;
  const int tx = px + H, ty = py + H;
  const int32_t hc = th[tx * TS + ty];
  const int64_t c = (int64_t)gx * a.ny + gy;
  uint8_t fl = a.flags[c];
  float slope = __uint_as_float(kQNaN), rough = __uint_as_float(kQNaN);
  if (hc != INT32_MIN) {
    int32_t n = 0, sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
    int64_t sz = 0, sxz = 0, syz = 0, szz = 0;
    for (int dx = -h; dx <= h; dx++)
      for (int dy = -h; dy <= h; dy++) {
        const int32_t v = th[(tx + dx) * TS + ty + dy];
        if (v == INT32_MIN) continue;
        const int64_t dz = (int64_t)v - hc;
        n++;
        sx += dx;
        sy += dy;
        sxx += dx * dx;
        syy += dy * dy;
        sxy += dx * dy;
        sz += dz;
        sxz += dx * dz;
        syz += dy * dz;
        szz += dz * dz;
      }
    // adjugate of M = [[sxx sxy sx] [sxy syy sy] [sx sy n]] (symmetric)
    const int64_t c00 = (int64_t)syy * n - (int64_t)sy * sy;
    const int64_t c01 = (int64_t)sy * sx - (int64_t)sxy * n;
    const int64_t c02 = (int64_t)sxy * sy - (int64_t)syy * sx;
    const int64_t c11 = (int64_t)sxx * n - (int64_t)sx * sx;
    const int64_t c12 = (int64_t)sxy * sx - (int64_t)sxx * sy;
    const int64_t c22 = (int64_t)sxx * syy - (int64_t)sxy * sxy;
    const int64_t det = (int64_t)sxx * c00 + (int64_t)sxy * c01 + (int64_t)sx * c02;
    if (n >= 3 && det != 0) {
      const double inv = 1.0 / (double)det;
      const double bx = (double)sxz, by = (double)syz, bz = (double)sz;
      const double al = ((double)c00 * bx + (double)c01 * by + (double)c02 * bz) * inv;
      const double be = ((double)c01 * bx + (double)c11 * by + (double)c12 * bz) * inv;
      const double ga = ((double)c02 * bx + (double)c12 * by + (double)c22 * bz) * inv;
      // residual sum of squares of the least-squares plane: z.z - beta.(X^T z)
      // (integer sums exact; |dz| < 2^23 Q units as nz <= 128, so the double
      // cancellation error stays far below the roughness tolerance)
      const double ss = fmax((double)szz - (al * bx + be * by + ga * bz), 0.0);
      slope = (float)(sqrt(al * al + be * be) / 65536.0);
      rough = (float)(ss / (double)n * a.q2m * a.q2m);
      fl |= 32;
    }
  } else {
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    int found = 0;
    // cones 0/1: +x/-x (slices on staged rows), 2/3: +y/-y (staged columns)
    for (int cone = 0; cone < 4; cone++) {
      const bool alongx = cone < 2;
      const int dir = (cone & 1) ? -1 : 1;
      const int ctr = alongx ? tx : ty;        // coordinate that moves with d
      const int oth = alongx ? ty : tx;        // centre of the slice span
      const uint8_t* dist = alongx ? rdist : cdist;
      const int j = alongx ? py : px;
      // first ring holding a defined cell: four rings per round (independent
      // LDS reads; ring indexes clamped to D stay inside the staged tile)
      int d = 1;
      for (; d <= D; d += 4) {
        const int d1 = min(d + 1, D), d2 = min(d + 2, D), d3 = min(d + 3, D);
        const int b0 = dist[(ctr + dir * d) * TILE + j];
        const int b1 = dist[(ctr + dir * d1) * TILE + j];
        const int b2 = dist[(ctr + dir * d2) * TILE + j];
        const int b3 = dist[(ctr + dir * d3) * TILE + j];
        if (b0 <= d) break;
        if (b1 <= d1) { d = d1; break; }
        if (b2 <= d2) { d = d2; break; }
        if (b3 <= d3) { d = d3; break; }
      }
      if (d > D) continue;
      const int line = ctr + dir * d;
      const int s0 = oth - d, s1 = oth + d;
      const unsigned long long* L = (alongx ? rmask : cmask) + line * MW;
      for (int w = s0 >> 6; w <= (s1 >> 6); w++) {
        unsigned long long b = span_bits(L[w], w, s0, s1);
        while (b) {
          const int k = 64 * w + __ffsll((long long)b) - 1;
          b &= b - 1;
          const int32_t v = alongx ? th[line * TS + k] : th[k * TS + line];
          lo = min(lo, v);
          hi = max(hi, v);
          found++;
        }
      }
    }
    if (found >= 2 && (int64_t)hi - lo > a.tau_q) fl |= 16;
  }
  a.slope[c] = slope;
  a.rough[c] = rough;
  a.flags[c] = fl;
  }
}


// Lookup-table export.  Ranks follow window-local column order: pass 1 gives
// every local column its occupied-voxel count prefix within its group of 64
// columns and each group its total, pass 2 scans the group totals, pass 3
// writes the table and the data array region by region.
constexpr int kGroup = 64;

__device__ __forceinline__ void lut_count_body(const LutArgs& a, const int blk) {
  const int nx = a.d.nx, ny = a.d.ny;
  const int lane = __lane_id();
  const int c = blk * kBlock + threadIdx.x;
  int cnt = 0;
  if (c < nx * ny) {
    const int x = c / ny, y = c - x * ny;
    const int64_t scol = (int64_t)wrap_add(x + a.d.ro[0], nx) * ny + wrap_add(y + a.d.ro[1], ny);
    cnt = __popcll(a.occ[scol * a.d.W]);
    if (a.d.W > 1) cnt += __popcll(a.occ[scol * a.d.W + 1]);
  }
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(incl, o);
    if (lane >= o) incl += u;
  }
  if (c < nx * ny) a.colpre[c] = incl - cnt;
  const int g = c >> 6;
  if (lane == 63 && g * kGroup < nx * ny) a.block_base[g] = incl;
}


// Pass 2 (one block): exclusive scan of the group counts; writes M.
template <int NT>
__device__ __forceinline__ void lut_scan_body(int32_t* base, const int nb, int64_t* n_occupied) {
  __shared__ int64_t wsum[NT / 64];
  const int t = threadIdx.x;
  const int per = (nb + NT - 1) / NT;
  const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
  // the thread's counts in chunks of 8 loads in flight (clamped in-bounds
  // loads, masked sums); the first chunk stays in registers for the writes
  constexpr int kChunk = 8;
  int32_t v0[kChunk];
  int64_t s = 0;
  for (int c = b0; c < b1; c += kChunk) {
    int32_t v[kChunk];
#pragma unroll
    for (int k = 0; k < kChunk; k++) v[k] = base[min(c + k, nb - 1)];
#pragma unroll
    for (int k = 0; k < kChunk; k++) {
      if (c + k < b1) s += v[k];
      if (c == b0) v0[k] = v[k];
    }
  }
  const int lane = __lane_id(), w = t >> 6;
  int64_t v = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int k = 0; k < NT / 64; k++) {
      const int64_t q = wsum[k];
      wsum[k] = acc;
      acc += q;
    }
    *n_occupied = acc;
  }
  __syncthreads();
  int64_t run = wsum[w] + v - s;  // exclusive prefix of this thread's range
#pragma unroll
  for (int k = 0; k < kChunk; k++) {
    if (b0 + k < b1) {
      base[b0 + k] = (int32_t)run;
      run += v0[k];
    }
  }
  for (int b = b0 + kChunk; b < b1; b++) {
    const int32_t q = base[b];
    base[b] = (int32_t)run;
    run += q;
  }
}


// Pass 3: block = a storage region of 4 x 16 columns (four 4 x 4 bricks,
// contiguous in memory).  The passes of the region are read in storage order
// (16-byte loads, all of a thread's loads in flight before its LDS stores)
// into LDS rows in window-local z order.  The occupied voxels' records are
// written one thread per voxel (the region's occupied voxels are numbered
// column by column, so a voxel's rank is its column base plus its number
// within the column, and every gather is issued at once).  Then every lane
// writes four consecutive table entries of one column (a transpose through
// LDS keeps both sides coalesced; one 16-byte LDS read and one 16-byte store
// per lane).
constexpr int kRegCols = 64;
constexpr int kLutLoads = 4;  // 16-byte region loads per thread per batch

// LDS row stride of a column's passes: a multiple of 4 words.
__host__ __device__ __forceinline__ int lut_row(int nz) { return ((nz + 3) & ~3) + 4; }

__device__ __forceinline__ void lut_write_body(const LutArgs& a, const uint32_t nz_magic,
                                               const int bxr, const int byr) {
  extern __shared__ __attribute__((aligned(16))) int32_t lpass[];  // [64][lut_row(nz)]
  __shared__ unsigned long long slo[kRegCols], shi[kRegCols];
  __shared__ int32_t sbase[kRegCols], spre[kRegCols + 1];
  __shared__ int64_t scb[kRegCols], slut[kRegCols];
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, W = a.d.W, roz = a.d.ro[2];
  const int nzp = lut_row(nz);
  const int tid = threadIdx.x;
  // storage-order read of the region: 16-byte word k4 holds brick b, level
  // zs, brick row iy (k4 = 4 (b nz + zs) + iy), voxels ix = 0..3
  const int nbricks = min(4, a.d.nby - 4 * byr);
  const int nv4 = nbricks * nz * 4;
  const int4* __restrict__ src = (const int4*)(a.passes + col_base(a.d, 4 * bxr, 16 * byr));
  for (int k0 = 0; k0 < nv4; k0 += kLutLoads * kBlock) {
    int4 v[kLutLoads];
#pragma unroll
    for (int u = 0; u < kLutLoads; u++) {
      // clamped, not skipped: every lane loads (in bounds), the stores below
      // skip the words past the region
      v[u] = src[min(k0 + u * kBlock + tid, nv4 - 1)];
    }
    if (k0 == 0 && tid < kRegCols) {
      // wave 0, after the first region loads are issued: the region's columns
      // (masks, rank bases, occupied-count prefix)
      Mask128 m = {0ull, 0ull};
      int32_t base = 0;
      int64_t cb = -1, lrow = 0;
      const int sx = 4 * bxr + (tid >> 4), sy = 16 * byr + (tid & 15);
      if (sx < nx && sy < ny) {
        const int x = sx - a.d.ro[0] + (sx < a.d.ro[0] ? nx : 0);
        const int y = sy - a.d.ro[1] + (sy < a.d.ro[1] ? ny : 0);
        const int c = x * ny + y;
        base = a.block_base[c >> 6] + a.colpre[c];
        m = local_mask(a.occ, (int64_t)sx * ny + sy, W, nz, roz);
        cb = col_base(a.d, sx, sy);
        lrow = (int64_t)c * nz;
      }
      const int cnt = __popcll(m.lo) + __popcll(m.hi);
      int incl = cnt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (tid >= o) incl += y;
      }
      slo[tid] = m.lo;
      shi[tid] = m.hi;
      sbase[tid] = base;
      scb[tid] = cb;
      slut[tid] = lrow;
      spre[tid] = incl - cnt;
      if (tid == kRegCols - 1) spre[kRegCols] = incl;
    }
#pragma unroll
    for (int u = 0; u < kLutLoads; u++) {
      const int k4 = k0 + u * kBlock + tid;
      if (k4 < nv4) {
        const int bz = k4 >> 2, iy = k4 & 3;
        const int b = nz == 1 ? bz : (int)__umulhi((uint32_t)bz, nz_magic);
        const int zs = bz - b * nz;
        const int lz = zs >= roz ? zs - roz : zs - roz + nz;
        int32_t* row = lpass + (4 * b + iy) * nzp + lz;  // slot = 16 ix + 4 b + iy
        row[0] = v[u].x;
        row[16 * nzp] = v[u].y;
        row[32 * nzp] = v[u].z;
        row[48 * nzp] = v[u].w;
      }
    }
  }
  __syncthreads();
  // records of the occupied voxels: voxel o of the region lies in the column t
  // with spre[t] <= o < spre[t + 1], at the set bit of rank o - spre[t]
  const int nocc = spre[kRegCols];
  for (int o = tid; o < nocc; o += kBlock) {
    int t = 0;
#pragma unroll
    for (int step = kRegCols / 2; step >= 1; step >>= 1)
      if (spre[t + step] <= o) t += step;
    const int r = o - spre[t];
    const int32_t rank = sbase[t] + r;
    if (rank < a.cap) {
      const int z = select_bit(Mask128{slo[t], shi[t]}, r);
      const int64_t idx = scb[t] + ((int64_t)wrap_add(z + roz, nz) << 4);
      map_voxel_t d;
      d.hits = a.hits[idx];
      d.passes = lpass[t * nzp + z];
      d.min_qz = a.minqz[idx];
      a.data[rank] = d;
    }
  }
  // items (column t, quad q): window-local z = 4q .. 4q+3; qs quads per column
  // rounded up to a power of two so that t and q are shifts
  const int nq = (nz + 3) >> 2;
  const int qsh = nq > 1 ? 32 - __clz(nq - 1) : 0;
  const bool vec = (nz & 3) == 0 && ((uintptr_t)a.lut & 15) == 0;
  for (int i = tid; i < (kRegCols << qsh); i += kBlock) {
    const int t = i >> qsh, q = i & ((1 << qsh) - 1);
    if (q >= nq || scb[t] < 0) continue;
    const Mask128 mt = {slo[t], shi[t]};
    const int z0 = 4 * q;
    const int4 pv = *(const int4*)(lpass + t * nzp + z0);
    const int32_t p4[4] = {pv.x, pv.y, pv.z, pv.w};
    int32_t rank = sbase[t] + rank_below(mt, z0);
    int32_t v[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int z = z0 + e;
      const bool occ = z < nz && test_bit(mt, z);
      v[e] = occ ? rank : -1 - p4[e];
      rank += occ;
    }
    // the table is written once and not read back here: streaming stores
    int32_t* __restrict__ lut = a.lut + slut[t] + z0;
    if (vec) {
      typedef int32_t v4i __attribute__((ext_vector_type(4)));
      const v4i vv = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(vv, (v4i*)lut);
    } else {
#pragma unroll
      for (int e = 0; e < 4; e++)
        if (z0 + e < nz) __builtin_nontemporal_store(v[e], lut + e);
    }
  }
}

}  // namespace
}  // namespace gvom
