// Export kernels: the per-column reductions and the 2D maps of Sec. III-D of
// arXiv 2109.13176, the Sec. III-A lookup table / data array, and its import.
#include <math.h>

#include "export_body.h"

namespace gvom {

namespace {

__global__ __launch_bounds__(kBlock) void k_column(ColumnArgs a) { column_body(a, blockIdx.x); }

template <int NT, int TILE>
__global__ __launch_bounds__(NT) void k_surface(SurfaceArgs a, int H) {
  surface_body<NT, TILE>(a, H, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBlock) void k_lut_count(LutArgs a) { lut_count_body(a, blockIdx.x); }

__global__ __launch_bounds__(1024) void k_lut_scan(int32_t* base, int nb, int64_t* n_occupied) {
  lut_scan_body<1024>(base, nb, n_occupied);
}

__global__ __launch_bounds__(kBlock) void k_lut_write(LutArgs a, uint32_t nz_magic) {
  lut_write_body(a, nz_magic, blockIdx.x, blockIdx.y);  // brick row, group of 4 bricks
}

// Density of every voxel (the voxel-map output, Fig. 1), in window-local
// table order: the storage region of the table export (4 x 16 columns) is
// read in storage order (16-byte loads, all of a thread's loads in flight
// before its LDS stores), each voxel's density computed there and kept in
// LDS rows in window-local z order; then every lane writes four consecutive
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
  // 16-byte word k4 of the region: brick b, level zs, brick row iy
  // (k4 = 4 (b nz + zs) + iy), voxels ix = 0..3 (slot 16 ix + 4 b + iy)
  const int nbricks = min(4, a.d.nby - 4 * byr);
  const int64_t r0 = col_base(a.d, 4 * bxr, 16 * byr);
  const int nv4 = nbricks * nz * 4;
  const int4* __restrict__ hsrc = (const int4*)(a.hits + r0);
  const int4* __restrict__ psrc = (const int4*)(a.passes + r0);
  for (int k0 = 0; k0 < nv4; k0 += kLutLoads * kBlock) {
    int4 hv[kLutLoads], pv[kLutLoads];
#pragma unroll
    for (int u = 0; u < kLutLoads; u++) {
      // clamped, not skipped: every lane loads (in bounds), the stores below
      // skip the words past the region
      const int k4 = min(k0 + u * kBlock + (int)threadIdx.x, nv4 - 1);
      hv[u] = hsrc[k4];
      pv[u] = psrc[k4];
    }
#pragma unroll
    for (int u = 0; u < kLutLoads; u++) {
      const int k4 = k0 + u * kBlock + threadIdx.x;
      if (k4 < nv4) {
        const int bz = k4 >> 2, iy = k4 & 3;
        const int b = nz == 1 ? bz : (int)__umulhi((uint32_t)bz, nz_magic);
        const int zs = bz - b * nz;
        const int lz = zs >= roz ? zs - roz : zs - roz + nz;
        const int32_t h4[4] = {hv[u].x, hv[u].y, hv[u].z, hv[u].w};
        const int32_t p4[4] = {pv[u].x, pv[u].y, pv[u].z, pv[u].w};
#pragma unroll
        for (int ix = 0; ix < 4; ix++) {
          const int32_t h = h4[ix], p = p4[ix];
          float v;
          if (h >= 1) v = (float)((double)h / ((double)h + (double)p));
          else v = p >= 1 ? 0.0f : __uint_as_float(kQNaN);
          lden[(16 * ix + 4 * b + iy) * nzp + lz] = v;
        }
      }
    }
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

// ---- batches: persistent grids over the virtual blocks of all maps
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

// The maps whose surface tile is TILE (index ti of pre_surf): tile 32 on
// 1,024-thread blocks, tile 16 on 256-thread blocks.
template <int NT, int TILE, int ti>
__global__ __launch_bounds__(NT) void k_b_surface(const BatchTables* __restrict__ t,
                                                  unsigned long long* stamps) {
  const int n = t->st.nmaps;
  const int32_t* pre = t->st.pre_surf[ti];
  const int total = pre[n];
  Stamper sp;
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map_e(pre, n, vb);
    const int tile = vb - pre[m];
    const int ty = t->st.surf_tiles_y[m];
    surface_body<NT, TILE>(t->sur[m], t->st.surf_H[m], tile / ty, tile % ty);
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
    lut_scan_body<1024>(t->lut[m].block_base, t->st.lut_groups[m], t->lut[m].n_occupied);
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
    hipError_t e = hipFuncSetAttribute((const void*)k_b_surface<kSurfThreads, kTile, 1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)g.surf_lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_b_surface<256, 16, 0>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.surf_lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_b_column, dim3(g.col), dim3(kBlock), 0, s, tab);
  hipLaunchKernelGGL((k_b_surface<256, 16, 0>), dim3(g.surf16), dim3(256), g.surf_lds, s, tab,
                     stamps);
  hipLaunchKernelGGL((k_b_surface<kSurfThreads, kTile, 1>), dim3(g.surf), dim3(kSurfThreads),
                     g.surf_lds, s, tab, stamps);
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

size_t surface_lds(int H, int tile) {
  const int T = tile + 2 * H;
  const int MW = (T + 63) / 64;
  return (size_t)((T * surface_stride(T) + 1) & ~1) * 4 + 2 * (size_t)T * MW * 8 +
         2 * (size_t)T * tile;
}

size_t lut_lds(int nz) { return (size_t)kRegCols * lut_row(nz) * 4; }

uint32_t nz_magic(int nz) {
  return nz > 1 ? (uint32_t)((((uint64_t)1 << 32) + (uint64_t)nz - 1) / (uint64_t)nz) : 0u;
}

// tile 32: one pixel per thread (1,024-thread blocks); tile 16: 256 threads
template <int NT, int TILE>
hipError_t launch_surface_t(const SurfaceArgs& a, hipStream_t s) {
  const int H = a.search_d > a.half_fit ? a.search_d : a.half_fit;
  const int T = TILE + 2 * H;
  const int MW = (T + 63) / 64;
  if (MW > kMaxMaskWords) return hipErrorInvalidValue;
  const size_t lds = surface_lds(H, TILE);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_surface<NT, TILE>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 g((a.nx + TILE - 1) / TILE, (a.ny + TILE - 1) / TILE);
  hipLaunchKernelGGL((k_surface<NT, TILE>), g, dim3(NT), lds, s, a, H);
  return hipGetLastError();
}

hipError_t launch_surface(const SurfaceArgs& a, int tile, hipStream_t s) {
  return tile == 16 ? launch_surface_t<256, 16>(a, s) : launch_surface_t<kSurfThreads, kTile>(a, s);
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
