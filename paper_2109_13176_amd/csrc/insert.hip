// Scan insertion kernels: transform + return binning + exact integer ray
// traversal (Sec. III-C of arXiv 2109.13176), and the slab clears that move
// the toroidal window.
#include <math.h>

#include "insert_body.h"

namespace gvom {

namespace {



template <bool DISTINCT>
__global__ __launch_bounds__(kRayBlock) void k_rays(InsertArgs a) {
  rays_body<DISTINCT>(a, blockIdx.x);
}

template <bool DISTINCT>
__global__ __launch_bounds__(kTraceBlock, kTraceWavesPerSimd) void k_trace(InsertArgs a) {
  __shared__ int32_t box_cnt[kBoxCells];
  __shared__ WaveTable wtab[kTraceBlock / 64];
  trace_body<DISTINCT, true, kTraceBlock>(a, blockIdx.x, gridDim.x, box_cnt, wtab);
}

template <bool DISTINCT>
__global__ __launch_bounds__(kBlock) void k_box_fold(InsertArgs a) {
  box_fold_body<DISTINCT>(a, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBlock) void k_clear(ClearArgs a) {
  clear_body(a, (int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock);
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
                                                    unsigned long long* stamps) {
  const int n = t->st.nmaps;
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  if (gid == 0) stamps[0] = wall_clock64();
  constexpr int kWords = 8 + kStripes;
  for (int64_t i = gid; i < (int64_t)n * kWords; i += stride) t->ins[i / kWords].stats[i % kWords] = 0;
  for (int64_t i = gid; i < n; i += stride) stamps[1 + i] = 0;  // per-map completion maxima
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

__global__ __launch_bounds__(kTraceBlock, kTraceWavesPerSimd) void k_b_trace(
    const BatchTables* __restrict__ t) {
  __shared__ int32_t box_cnt[kBoxCells];
  __shared__ WaveTable wtab[kTraceBlock / 64];
  const int n = t->st.nmaps;
  const int total = t->st.pre_trace[n];
  for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
    const int m = find_map(t->st.pre_trace, n, vb);
    trace_body<false, true, kTraceBlock>(t->ins[m], vb - t->st.pre_trace[m],
                                         t->ins[m].trace_blocks, box_cnt, wtab);
    __syncthreads();
  }
}

// Sensor-box folds of every map of the batch: block b = map b / F, fold block
// b mod F (F = kFoldCellBlocks x kFoldGroups).
__global__ __launch_bounds__(kBlock) void k_b_box_fold(const BatchTables* __restrict__ t) {
  constexpr int F = kFoldCellBlocks * kFoldGroups;
  const int m = blockIdx.x / F, f = blockIdx.x - m * F;
  if (m >= t->st.nmaps) return;
  box_fold_body<false>(t->ins[m], f % kFoldCellBlocks, f / kFoldCellBlocks);
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
                               unsigned long long* stamps, hipStream_t s) {
  hipLaunchKernelGGL(k_b_clear, dim3(g.clear), dim3(kBlock), 0, s, tab, stamps);
  hipLaunchKernelGGL(k_b_rays, dim3(g.rays), dim3(kRayBlock), 0, s, tab);
  hipLaunchKernelGGL(k_b_trace, dim3(g.trace), dim3(kTraceBlock), 0, s, tab);
  hipLaunchKernelGGL(k_b_box_fold, dim3(g.fold), dim3(kBlock), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

int64_t max_segments(const Dims& d, int32_t seg_len) {
  int32_t m = d.nx > d.ny ? d.nx : d.ny;
  if (d.nz > m) m = d.nz;
  return (m - 1) / seg_len + 1;
}

hipError_t launch_rays(const InsertArgs& a, bool distinct, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int g = (a.n + kRayBlock - 1) / kRayBlock;
  if (distinct)
    hipLaunchKernelGGL(k_rays<true>, dim3(g), dim3(kRayBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_rays<false>, dim3(g), dim3(kRayBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_trace(const InsertArgs& a, bool distinct, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  if (!a.box_rep || a.trace_blocks < 1) return hipErrorInvalidValue;
  const dim3 fb(kFoldCellBlocks, kFoldGroups);
  if (distinct) {
    hipLaunchKernelGGL(k_trace<true>, dim3(a.trace_blocks), dim3(kTraceBlock), 0, s, a);
    hipLaunchKernelGGL(k_box_fold<true>, dim3(fb), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_trace<false>, dim3(a.trace_blocks), dim3(kTraceBlock), 0, s, a);
    hipLaunchKernelGGL(k_box_fold<false>, dim3(fb), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

int box_fold_blocks() { return kFoldCellBlocks * kFoldGroups; }
int box_fold_groups() { return kFoldGroups; }
// Sums the ray pass's per-block counters (4 per block) into out[0..3]: one
// block, each thread a strided share of the blocks, then a fixed-order sum
// over the threads (no atomics).
__global__ __launch_bounds__(kBlock) void k_sum_ray_parts(const unsigned long long* parts,
                                                          int64_t nblocks,
                                                          unsigned long long* out) {
  __shared__ unsigned long long s[4][kBlock];
  unsigned long long c[4] = {0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nblocks; b += kBlock)
#pragma unroll
    for (int k = 0; k < 4; k++) c[k] += parts[4 * b + k];
#pragma unroll
  for (int k = 0; k < 4; k++) s[k][threadIdx.x] = c[k];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int k = 0; k < 4; k++) s[k][threadIdx.x] += s[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

hipError_t launch_sum_ray_parts(const unsigned long long* parts, int64_t nblocks,
                                unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_ray_parts, dim3(1), dim3(kBlock), 0, s, parts, nblocks, out);
  return hipGetLastError();
}


}  // namespace gvom
