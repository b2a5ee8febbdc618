// Export kernels: the per-column reductions and the 2D maps of Sec. III-D of
// arXiv 2109.13176, the Sec. III-A lookup table / data array, and its import.
#include <math.h>

#include "gvom_internal.h"

namespace gvom {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kQNaN = 0x7FC00000u;

__device__ __forceinline__ int32_t wrap_add(int32_t s, int32_t n) { return s >= n ? s - n : s; }

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
    for (int z = zlo; z <= zhi; z++) {
      if (!test_bit(m, z)) continue;
      const int64_t e = base + (wrap_add(z + a.d.ro[2], nz) << 4);
      const int32_t h = a.hits[e];
      sh += h;
      sa += (int64_t)h + a.passes[e];
      cnt++;
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

__global__ __launch_bounds__(kBlock) void k_column(ColumnArgs a) { column_body(a, blockIdx.x); }

// 2D surface maps on tiles of kTile x kTile pixels (one pixel per thread)
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

__device__ __forceinline__ void surface_body(const SurfaceArgs& a, const int H, const int bx,
                                             const int by) {
  extern __shared__ int32_t lds[];
  const int T = kTile + 2 * H;          // staged tile edge
  const int TS = surface_stride(T);     // LDS row stride of th
  const int MW = (T + 63) >> 6;         // mask words per staged row / column
  int32_t* th = lds;                                                    // [T][TS]
  unsigned long long* rmask = (unsigned long long*)(lds + ((T * TS + 1) & ~1));  // [T][MW]
  unsigned long long* cmask = rmask + T * MW;                            // [T][MW]
  uint8_t* rdist = (uint8_t*)(cmask + T * MW);  // [T][kTile]: row r, tile column j
  uint8_t* cdist = rdist + T * kTile;           // [T][kTile]: column c, tile row i
  const int gx0 = bx * kTile - H, gy0 = by * kTile - H;
  const int lane = __lane_id(), wv = threadIdx.x >> 6;
  constexpr int kWaves = kSurfThreads / 64;
  // stage the heights row by row (a wave per row, lanes along y); the
  // ballot of each 64-cell piece is that row's mask word
  for (int r = wv; r < T; r += kWaves) {
    const int gx = gx0 + r;
    const bool rowok = gx >= 0 && gx < a.nx;
    for (int w = 0; w < MW; w++) {
      const int k = 64 * w + lane;
      const int gy = gy0 + k;
      int32_t v = INT32_MIN;
      if (k < T && rowok && gy >= 0 && gy < a.ny) v = a.hq[(int64_t)gx * a.ny + gy];
      if (k < T) th[r * TS + k] = v;
      const unsigned long long b = __ballot(v != INT32_MIN);
      if (lane == 0) rmask[r * MW + w] = b;
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
  for (int i = threadIdx.x; i < 2 * T * kTile; i += kSurfThreads) {
    const bool col = i >= T * kTile;
    const int ii = col ? i - T * kTile : i;
    const int line = ii / kTile, j = ii - line * kTile;
    const int dd = line_distance((col ? cmask : rmask) + line * MW, MW, T, H + j);
    (col ? cdist : rdist)[ii] = (uint8_t)dd;
  }

  // defined pixels (plane fit) and undefined ones (cone search) go to
  // separate waves: the block's pixels are listed defined-first, ranks from
  // ballots (deterministic order)
  __shared__ int16_t order[kSurfThreads];
  __shared__ int wcnt[kWaves][2];
  {
    const int px = threadIdx.x / kTile, py = threadIdx.x - px * kTile;
    const int gx = bx * kTile + px, gy = by * kTile + py;
    const bool valid = gx < a.nx && gy < a.ny;
    const bool def = valid && th[(px + H) * TS + py + H] != INT32_MIN;
    const bool und = valid && !def;
    const unsigned long long bd = __ballot(def), bu = __ballot(und);
    if (lane == 0) {
      wcnt[wv][0] = __popcll(bd);
      wcnt[wv][1] = __popcll(bu);
    }
    __syncthreads();
    int pd = 0, pu = 0;
    for (int w = 0; w < wv; w++) {
      pd += wcnt[w][0];
      pu += wcnt[w][1];
    }
    const int below_d = __builtin_amdgcn_mbcnt_hi((uint32_t)(bd >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bd, 0));
    const int below_u = __builtin_amdgcn_mbcnt_hi((uint32_t)(bu >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)bu, 0));
    if (def) order[pd + below_d] = (int16_t)threadIdx.x;
    if (und) order[kSurfThreads - 1 - (pu + below_u)] = (int16_t)threadIdx.x;
  }
  __syncthreads();
  int nd = 0, nu = 0;
  for (int w = 0; w < kWaves; w++) {
    nd += wcnt[w][0];
    nu += wcnt[w][1];
  }
  int me;
  if ((int)threadIdx.x < nd) me = order[threadIdx.x];
  else if ((int)threadIdx.x >= kSurfThreads - nu) me = order[threadIdx.x];
  else return;
  const int px = me / kTile, py = me - px * kTile;
  const int gx = bx * kTile + px, gy = by * kTile + py;
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
        const int b0 = dist[(ctr + dir * d) * kTile + j];
        const int b1 = dist[(ctr + dir * d1) * kTile + j];
        const int b2 = dist[(ctr + dir * d2) * kTile + j];
        const int b3 = dist[(ctr + dir * d3) * kTile + j];
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

__global__ __launch_bounds__(kSurfThreads) void k_surface(SurfaceArgs a, int H) {
  surface_body(a, H, blockIdx.x, blockIdx.y);
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

__global__ __launch_bounds__(kBlock) void k_lut_count(LutArgs a) { lut_count_body(a, blockIdx.x); }

// Pass 2 (one block): exclusive scan of the group counts; writes M.
__device__ __forceinline__ void lut_scan_body(int32_t* base, const int nb, int64_t* n_occupied) {
  __shared__ int64_t wsum[16];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(t * per, nb), b1 = min(b0 + per, nb);
  int64_t s = 0;
  for (int b = b0; b < b1; b++) s += base[b];
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
    for (int k = 0; k < 16; k++) {
      const int64_t q = wsum[k];
      wsum[k] = acc;
      acc += q;
    }
    *n_occupied = acc;
  }
  __syncthreads();
  int64_t run = wsum[w] + v - s;  // exclusive prefix of this thread's range
  for (int b = b0; b < b1; b++) {
    const int32_t q = base[b];
    base[b] = (int32_t)run;
    run += q;
  }
}

__global__ __launch_bounds__(1024) void k_lut_scan(int32_t* base, int nb, int64_t* n_occupied) {
  lut_scan_body(base, nb, n_occupied);
}

// Pass 3: block = a storage region of 4 x 16 columns (four 4 x 4 bricks,
// contiguous in memory).  The passes of the region are read in storage order
// into LDS rows in window-local z order, then every lane writes four
// consecutive table entries of one column (a transpose through LDS keeps both
// sides coalesced; one 16-byte LDS read and one 16-byte store per lane).
constexpr int kRegCols = 64;

// LDS row stride of a column's passes: a multiple of 4 words.
__host__ __device__ __forceinline__ int lut_row(int nz) { return ((nz + 3) & ~3) + 4; }

__device__ __forceinline__ void lut_write_body(const LutArgs& a, const uint32_t nz_magic,
                                               const int bxr, const int byr) {
  extern __shared__ __attribute__((aligned(16))) int32_t lpass[];  // [64][lut_row(nz)]
  __shared__ unsigned long long slo[kRegCols], shi[kRegCols];
  __shared__ int32_t sbase[kRegCols];
  __shared__ int64_t scb[kRegCols], slut[kRegCols];
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, W = a.d.W, roz = a.d.ro[2];
  const int nzp = lut_row(nz);
  if (threadIdx.x < kRegCols) {
    const int t = threadIdx.x;
    const int ix = t >> 4, jy = t & 15;
    const int sx = 4 * bxr + ix, sy = 16 * byr + jy;
    Mask128 m = {0ull, 0ull};
    int32_t base = 0;
    int64_t cb = -1, lrow = 0;
    if (sx < nx && sy < ny) {
      const int x = sx - a.d.ro[0] + (sx < a.d.ro[0] ? nx : 0);
      const int y = sy - a.d.ro[1] + (sy < a.d.ro[1] ? ny : 0);
      const int c = x * ny + y;
      m = local_mask(a.occ, (int64_t)sx * ny + sy, W, nz, roz);
      base = a.block_base[c >> 6] + a.colpre[c];
      cb = col_base(a.d, sx, sy);
      lrow = (int64_t)c * nz;
    }
    slo[t] = m.lo;
    shi[t] = m.hi;
    sbase[t] = base;
    scb[t] = cb;
    slut[t] = lrow;
  }
  // storage-order read of the region: brick b (0..3), level z, lane16 = 4 iy + ix
  const int nbricks = min(4, a.d.nby - 4 * byr);
  const int64_t r0 = col_base(a.d, 4 * bxr, 16 * byr);
  const int total = nbricks * nz * 16;
  const int32_t* __restrict__ passes = a.passes;
#pragma unroll 4
  for (int k = threadIdx.x; k < total; k += kBlock) {
    const int bz = k >> 4, l16 = k & 15;
    const int b = nz == 1 ? bz : (int)__umulhi((uint32_t)bz, nz_magic);
    const int zs = bz - b * nz;
    const int lz = zs >= roz ? zs - roz : zs - roz + nz;
    const int slot = (l16 & 3) * 16 + 4 * b + (l16 >> 2);
    lpass[slot * nzp + lz] = passes[r0 + k];
  }
  __syncthreads();
  // items (column t, quad q): window-local z = 4q .. 4q+3; qs quads per column
  // rounded up to a power of two so that t and q are shifts
  const int nq = (nz + 3) >> 2;
  const int qsh = nq > 1 ? 32 - __clz(nq - 1) : 0;
  const bool vec = (nz & 3) == 0 && ((uintptr_t)a.lut & 15) == 0;
  for (int i = threadIdx.x; i < (kRegCols << qsh); i += kBlock) {
    const int t = i >> qsh, q = i & ((1 << qsh) - 1);
    if (q >= nq || scb[t] < 0) continue;
    const Mask128 m = {slo[t], shi[t]};
    const int z0 = 4 * q;
    const int4 pv = *(const int4*)(lpass + t * nzp + z0);
    const int32_t p4[4] = {pv.x, pv.y, pv.z, pv.w};
    int32_t rank = sbase[t] + rank_below(m, z0);
    int32_t v[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int z = z0 + e;
      if (z < nz && test_bit(m, z)) {
        v[e] = rank;
        if (rank < a.cap) {
          const int64_t idx = scb[t] + ((int64_t)wrap_add(z + roz, nz) << 4);
          map_voxel_t d;
          d.hits = a.hits[idx];
          d.passes = p4[e];
          d.min_qz = a.minqz[idx];
          a.data[rank] = d;
        }
        rank++;
      } else {
        v[e] = -1 - p4[e];
      }
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

__global__ __launch_bounds__(kBlock) void k_lut_write(LutArgs a, uint32_t nz_magic) {
  lut_write_body(a, nz_magic, blockIdx.x, blockIdx.y);  // brick row, group of 4 bricks
}

// Density of every voxel (the voxel-map output, Fig. 1), in window-local
// table order: the storage region of the table export (4 x 16 columns) is
// read in storage order, each voxel's density computed there and kept in LDS
// rows in window-local z order; then every lane writes four consecutive
// densities of one column.
__global__ __launch_bounds__(kBlock) void k_density(DensityArgs a, uint32_t nz_magic) {
  extern __shared__ __attribute__((aligned(16))) float lden[];  // [64][lut_row(nz)]
  __shared__ int64_t sout[kRegCols];
  const int nx = a.d.nx, ny = a.d.ny, nz = a.d.nz, roz = a.d.ro[2];
  const int nzp = lut_row(nz);
  const int bxr = blockIdx.x, byr = blockIdx.y;
  if (threadIdx.x < kRegCols) {
    const int t = threadIdx.x;
    const int sx = 4 * bxr + (t >> 4), sy = 16 * byr + (t & 15);
    int64_t o = -1;
    if (sx < nx && sy < ny) {
      const int x = sx - a.d.ro[0] + (sx < a.d.ro[0] ? nx : 0);
      const int y = sy - a.d.ro[1] + (sy < a.d.ro[1] ? ny : 0);
      o = ((int64_t)x * ny + y) * nz;
    }
    sout[t] = o;
  }
  const int nbricks = min(4, a.d.nby - 4 * byr);
  const int64_t r0 = col_base(a.d, 4 * bxr, 16 * byr);
  const int total = nbricks * nz * 16;
  for (int k = threadIdx.x; k < total; k += kBlock) {
    const int bz = k >> 4, l16 = k & 15;
    const int b = nz == 1 ? bz : (int)__umulhi((uint32_t)bz, nz_magic);
    const int zs = bz - b * nz;
    const int lz = zs >= roz ? zs - roz : zs - roz + nz;
    const int slot = (l16 & 3) * 16 + 4 * b + (l16 >> 2);
    const int32_t h = a.hits[r0 + k], p = a.passes[r0 + k];
    float v;
    if (h >= 1) v = (float)((double)h / ((double)h + (double)p));
    else v = p >= 1 ? 0.0f : __uint_as_float(kQNaN);
    lden[slot * nzp + lz] = v;
  }
  __syncthreads();
  const int nq = (nz + 3) >> 2;
  const int qsh = nq > 1 ? 32 - __clz(nq - 1) : 0;
  const bool vec = (nz & 3) == 0 && ((uintptr_t)a.out & 15) == 0;
  for (int i = threadIdx.x; i < (kRegCols << qsh); i += kBlock) {
    const int t = i >> qsh, q = i & ((1 << qsh) - 1);
    if (q >= nq || sout[t] < 0) continue;
    const int z0 = 4 * q;
    float* __restrict__ out = a.out + sout[t] + z0;
    const float* src = lden + t * nzp + z0;
    if (vec) {
      typedef float v4f __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(*(const v4f*)src, (v4f*)out);
    } else {
      for (int e = 0; e < 4; e++)
        if (z0 + e < nz) __builtin_nontemporal_store(src[e], out + e);
    }
  }
}

// Costmap: one lane per pixel, the weighted layers added in a fixed order
// in binary32.
__global__ __launch_bounds__(kBlock) void k_costmap(CostArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const float sl = a.slope[i], ro = a.rough[i], de = a.density[i];
  const uint32_t f = a.flags[i];
  float c = 0.0f;
  if (!isnan(sl)) c = c + a.w[0] * sl;
  if (!isnan(ro)) c = c + a.w[1] * ro;
  if (!isnan(de)) c = c + a.w[2] * de;
  if (f & 2u) c = c + a.w[3];
  if (f & 4u) c = c + a.w[4];
  if (f & 8u) c = c + a.w[5];
  if (f & 16u) c = c + a.w[6];
  if (!(f & 1u)) c = c + a.w[7];
  a.cost[i] = c;
}

// Import: one wave per window-local column; lane = local z.
__global__ __launch_bounds__(kBlock) void k_import(Dims d, const int32_t* lut,
                                                   const map_voxel_t* data, int64_t n_data,
                                                   int32_t* hits, int32_t* passes,
                                                   int32_t* minqz, unsigned long long* occ,
                                                   int32_t* err) {
  const int lane = __lane_id();
  const int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  if (c >= (int64_t)nx * ny) return;
  const int x = (int)(c / ny), y = (int)(c - (int64_t)x * ny);
  const int sx = wrap_add(x + d.ro[0], nx), sy = wrap_add(y + d.ro[1], ny);
  const int64_t scol = (int64_t)sx * ny + sy;
  const int64_t cb = col_base(d, sx, sy);
  unsigned long long w0 = 0, w1 = 0;
  for (int zb = 0; zb < nz; zb += 64) {
    const int z = zb + lane;
    bool occd = false;
    if (z < nz) {
      const int32_t v = lut[c * nz + z];
      const int sz = wrap_add(z + d.ro[2], nz);
      const int64_t e = cb + ((int64_t)sz << 4);
      int32_t h = 0, p = 0, mq = INT32_MAX;
      if (v >= 0) {
        if (v < n_data && data[v].hits >= 1) {
          h = data[v].hits;
          p = data[v].passes;
          mq = data[v].min_qz;
          occd = true;
        } else {
          atomicOr(err, 1);
        }
      } else if (v == INT32_MIN) {
        atomicOr(err, 1);
      } else {
        p = -1 - v;
      }
      hits[e] = h;
      passes[e] = p;
      minqz[e] = mq;
      if (occd) {
        if (sz < 64) w0 |= 1ull << sz; else w1 |= 1ull << (sz - 64);
      }
    }
  }
  // combine the lanes' bits
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    w0 |= __shfl_xor(w0, o);
    w1 |= __shfl_xor(w1, o);
  }
  if (lane == 0) {
    occ[scol * d.W] = w0;
    if (d.W > 1) occ[scol * d.W + 1] = w1;
  }
}

// ---------------------------------------------------------------------------
// Batched stages (see insert.hip): persistent grids over the virtual blocks of
// all maps.  The map's last stage stamps its completion time.
__device__ __forceinline__ int find_map_e(const int32_t* pre, int n, int vb) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= vb) lo = mid; else hi = mid;
  }
  return lo;
}

// Completion time of map m: the latest end of its last-stage blocks, kept by
// a fire-and-forget 64-bit max (no fence: only the clock value matters).  A
// persistent block folds consecutive virtual blocks of one map into one
// update, made when it moves on to another map and at its end.
struct Stamper {
  int m = -1;
  unsigned long long end = 0;
  // after the (synchronised) virtual block of map mm; counts only if `last`
  __device__ __forceinline__ void done(int mm, bool last, unsigned long long* stamps) {
    if (threadIdx.x != 0) return;
    if (mm != m) flush(stamps);
    if (last) {
      m = mm;
      end = wall_clock64();
    }
  }
  __device__ __forceinline__ void flush(unsigned long long* stamps) {
    if (threadIdx.x == 0 && m >= 0) atomicMax(&stamps[1 + m], end);
    m = -1;
  }
};

__global__ __launch_bounds__(kBlock) void k_b_column(const BatchTables* __restrict__ t) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_col[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(t->st.pre_col, n, vb);
    column_body(t->col[m], vb - t->st.pre_col[m]);
  }
}

__global__ __launch_bounds__(kSurfThreads) void k_b_surface(const BatchTables* __restrict__ t,
                                                            unsigned long long* stamps) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_surf[n];
  Stamper sp;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(t->st.pre_surf, n, vb);
    const int tile = vb - t->st.pre_surf[m];
    const int ty = t->st.surf_tiles_y[m];
    surface_body(t->sur[m], t->st.surf_H[m], tile / ty, tile % ty);
    __syncthreads();
    sp.done(m, !t->st.last_is_lut[m], stamps);
  }
  sp.flush(stamps);
}

__global__ __launch_bounds__(kBlock) void k_b_lut_count(const BatchTables* __restrict__ t) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_lcount[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(t->st.pre_lcount, n, vb);
    lut_count_body(t->lut[m], vb - t->st.pre_lcount[m]);
  }
}

__global__ __launch_bounds__(1024) void k_b_lut_scan(const BatchTables* __restrict__ t) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_lscan[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(t->st.pre_lscan, n, vb);
    lut_scan_body(t->lut[m].block_base, t->st.lut_groups[m], t->lut[m].n_occupied);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_b_lut_write(const BatchTables* __restrict__ t,
                                                        unsigned long long* stamps) {
  const int n = t->st.nmaps;
  const int total = t->st.pre_lwrite[n];
  Stamper sp;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(t->st.pre_lwrite, n, vb);
    const int b = vb - t->st.pre_lwrite[m];
    const int by = t->st.lw_by[m];
    lut_write_body(t->lut[m], t->st.nz_magic[m], b / by, b % by);
    __syncthreads();
    sp.done(m, true, stamps);
  }
  sp.flush(stamps);
}

}  // namespace

hipError_t launch_batch_export(const BatchTables* tab, const BatchGrid& g,
                               unsigned long long* stamps, hipStream_t s) {
  if (g.surf_lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_b_surface,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)g.surf_lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_b_column, dim3(g.col), dim3(kBlock), 0, s, tab);
  hipLaunchKernelGGL(k_b_surface, dim3(g.surf), dim3(kSurfThreads), g.surf_lds, s, tab, stamps);
  hipLaunchKernelGGL(k_b_lut_count, dim3(g.lcount), dim3(kBlock), 0, s, tab);
  hipLaunchKernelGGL(k_b_lut_scan, dim3(g.lcount), dim3(1024), 0, s, tab);
  hipLaunchKernelGGL(k_b_lut_write, dim3(g.lwrite), dim3(kBlock), g.lut_lds, s, tab, stamps);
  return hipGetLastError();
}

hipError_t launch_column(const ColumnArgs& a, hipStream_t s) {
  const int C = a.d.nx * a.d.ny;
  hipLaunchKernelGGL(k_column, dim3((C + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int surface_tile() { return kTile; }

size_t surface_lds(int H) {
  const int T = kTile + 2 * H;
  const int MW = (T + 63) / 64;
  return (size_t)((T * surface_stride(T) + 1) & ~1) * 4 + 2 * (size_t)T * MW * 8 +
         2 * (size_t)T * kTile;
}

size_t lut_lds(int nz) { return (size_t)kRegCols * lut_row(nz) * 4; }

uint32_t nz_magic(int nz) {
  return nz > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)nz - 1) / (uint64_t)nz) : 0u;
}

hipError_t launch_surface(const SurfaceArgs& a, hipStream_t s) {
  const int H = a.search_d > a.half_fit ? a.search_d : a.half_fit;
  const int T = kTile + 2 * H;
  const int MW = (T + 63) / 64;
  if (MW > kMaxMaskWords) return hipErrorInvalidValue;
  const size_t lds = surface_lds(H);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_surface,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 g((a.nx + kTile - 1) / kTile, (a.ny + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_surface, g, dim3(kSurfThreads), lds, s, a, H);
  return hipGetLastError();
}

hipError_t launch_lut(const LutArgs& a, bool counted, hipStream_t s) {
  const int C = a.d.nx * a.d.ny;
  const int ng = (C + kGroup - 1) / kGroup;
  // b / nz == umulhi(b, ceil(2^32 / nz)) for every b < 2^20 (here b < 4 * 128)
  const uint32_t magic =
      a.d.nz > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)a.d.nz - 1) / (uint64_t)a.d.nz) : 0u;
  const size_t lds = lut_lds(a.d.nz);
  if (!counted)
    hipLaunchKernelGGL(k_lut_count, dim3((C + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_lut_scan, dim3(1), dim3(1024), 0, s, a.block_base, ng, a.n_occupied);
  dim3 g((a.d.nx + 3) / 4, (a.d.nby + 3) / 4);
  hipLaunchKernelGGL(k_lut_write, g, dim3(kBlock), lds, s, a, magic);
  return hipGetLastError();
}

hipError_t launch_density(const DensityArgs& a, hipStream_t s) {
  dim3 g((a.d.nx + 3) / 4, (a.d.nby + 3) / 4);
  hipLaunchKernelGGL(k_density, g, dim3(kBlock), lut_lds(a.d.nz), s, a, nz_magic(a.d.nz));
  return hipGetLastError();
}

hipError_t launch_costmap(const CostArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_costmap, dim3((unsigned)((a.n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     a);
  return hipGetLastError();
}

hipError_t launch_scan_i32(int32_t* base, int nb, int64_t* total, hipStream_t s) {
  hipLaunchKernelGGL(k_lut_scan, dim3(1), dim3(1024), 0, s, base, nb, total);
  return hipGetLastError();
}

hipError_t launch_import(const Dims& d, const int32_t* lut, const map_voxel_t* data,
                         int64_t n_data, int32_t* hits, int32_t* passes, int32_t* minqz,
                         unsigned long long* occ, int32_t* err, hipStream_t s) {
  const int64_t threads = (int64_t)d.nx * d.ny * 64;
  hipLaunchKernelGGL(k_import, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, d, lut, data, n_data, hits, passes, minqz, occ, err);
  return hipGetLastError();
}

}  // namespace gvom
