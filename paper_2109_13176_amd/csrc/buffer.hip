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
  const unsigned long long* occ;
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
// Every passes word is zeroed; hits and lowest return only where occupied
// (they are empty elsewhere).
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
      if (a.d.W > 1) hi = a.occ[col + 1];
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
      const int64_t s = s_b + 16 * z + 4 * q;
      const int4 p = *(const int4*)(a.passes + s);
      const int32_t pv[4] = {p.x, p.y, p.z, p.w};
      int32_t v[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        if ((bits >> e) & 1u) {
          if (rank < a.cap) {
            map_voxel_t dv;
            dv.hits = a.hits[s + e];
            dv.passes = pv[e];
            dv.min_qz = a.minqz[s + e];
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
      *(int4*)(a.passes + s) = make_int4(0, 0, 0, 0);
    }
    __syncthreads();  // wtot is rewritten by the next round
  }
}

__device__ __forceinline__ int32_t ring_to_local(int32_t s, int32_t ro, int32_t n) {
  const int32_t l = s - ro;
  return l < 0 ? l + n : l;
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
    const int sy = 4 * by + q;
    const int32_t gy = a.O[1] + ring_to_local(sy, a.d.ro[1], ny);
    const int32_t gz = a.O[2] + ring_to_local(z, a.d.ro[2], nz);
    int32_t gx[4];
    bool valid[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const int sx = 4 * bx + e;
      valid[e] = sx < nx && sy < ny;
      gx[e] = a.O[0] + ring_to_local(sx, a.d.ro[0], nx);
    }
    int32_t h[4] = {0, 0, 0, 0}, p[4] = {0, 0, 0, 0};
    int32_t mq[4] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    for (int k = 0; k < a.k; k++) {
      if ((uint32_t)(gy - a.org[k][1]) >= (uint32_t)ny ||
          (uint32_t)(gz - a.org[k][2]) >= (uint32_t)nz)
        continue;
      bool in[4], any = false;
#pragma unroll
      for (int e = 0; e < 4; e++) {
        in[e] = valid[e] && (uint32_t)(gx[e] - a.org[k][0]) < (uint32_t)nx;
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
    *(int4*)(a.hits + s) = make_int4(h[0], h[1], h[2], h[3]);
    *(int4*)(a.passes + s) = make_int4(p[0], p[1], p[2], p[3]);
    *(int4*)(a.minqz + s) = make_int4(mq[0], mq[1], mq[2], mq[3]);
#pragma unroll
    for (int e = 0; e < 4; e++) {
      if (h[e] > 0) {
        const int j = 4 * q + e;
        if (z < 64) atomicOr(&mlo[j], 1ull << z);
        else atomicOr(&mhi[j], 1ull << (z - 64));
      }
    }
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

int64_t n_bricks(const Dims& d) { return (int64_t)((d.nx + 3) / 4) * d.nby; }

}  // namespace

}  // namespace gvom

struct map_buffer_t {
  map_params_t p;
  int32_t depth;
  hipStream_t stream;           // producer stream: pushes run here
  map_t* prod;                  // producer map, empty between pushes
  struct Slot {
    int32_t* lut;
    map_voxel_t* data;
    int64_t cap;
    int32_t origin[3];
  };
  std::vector<Slot> slots;
  int32_t head;                 // slot of the next push
  int32_t count;                // buffered maps
  int32_t* brick_cnt;           // per brick: occupied voxels
  int32_t* group_cnt;           // per 16 bricks: occupied voxels, then their prefix
  int64_t* n_occ;               // [depth] occupied voxels per slot (device)
  hipEvent_t pushed;            // recorded after every push
  std::vector<hipEvent_t> pending;  // combines that may still read the slots
  std::vector<hipEvent_t> pool;
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
  for (hipEvent_t ev : b->pending) {
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
    b->pool.push_back(ev);
  }
  b->pending.clear();
  return e;
}

int32_t newest(const map_buffer_t* b) { return (b->head + b->depth - 1) % b->depth; }

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
  b->stream = (hipStream_t)stream;
  b->prod = prod;
  b->slots.assign(depth, map_buffer_t::Slot{nullptr, nullptr, 0, {0, 0, 0}});
  b->head = 0;
  b->count = 0;
  b->sticky = MAP_OK;
  const int64_t nb = gvom::n_bricks(prod->d);
  hipError_t e = hipMalloc((void**)&b->brick_cnt, (size_t)nb * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&b->group_cnt, (size_t)((nb + 15) / 16) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&b->n_occ, (size_t)depth * 8);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->pushed, hipEventDisableTiming);
  else b->pushed = nullptr;
  for (int i = 0; i < depth && e == hipSuccess; i++) {
    e = hipMalloc((void**)&b->slots[i].lut, (size_t)prod->d.vs * 4);
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
  for (hipEvent_t ev : b->pending) {
    (void)hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
  }
  for (hipEvent_t ev : b->pool) (void)hipEventDestroy(ev);
  for (auto& s : b->slots) {
    (void)hipFree(s.lut);
    (void)hipFree(s.data);
  }
  (void)hipFree(b->brick_cnt);
  (void)hipFree(b->group_cnt);
  (void)hipFree(b->n_occ);
  if (b->pushed) (void)hipEventDestroy(b->pushed);
  map_destroy(b->prod);
  (void)hipGetLastError();
  delete b;
  return MAP_OK;
}

int32_t map_buffer_reset(map_buffer_t* b) {
  if (!b) return MAP_E_INVALID;
  (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t ev : b->pending) {
    (void)hipEventSynchronize(ev);
    b->pool.push_back(ev);
  }
  b->pending.clear();
  (void)hipGetLastError();
  b->head = 0;
  b->count = 0;
  b->sticky = MAP_OK;
  return map_reset(b->prod);
}

int32_t map_buffer_push(map_buffer_t* b, const float* xyz_dev, int64_t n, const float pose[12],
                        uint32_t flags) {
  if (!b) return MAP_E_INVALID;
  if (b->sticky) return b->sticky;
  map_t* m = b->prod;
  // a scan that is not recentred takes the newest buffered window
  int32_t o[3];
  if (b->count > 0) {
    const map_buffer_t::Slot& nw = b->slots[newest(b)];
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
  map_buffer_t::Slot& s = b->slots[b->head];
  const int64_t need = n < m->d.vs ? (n > 0 ? n : 1) : m->d.vs;
  if (need > s.cap) {
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return buf_fail(b, e);
    const int64_t want = s.cap > 0 && need < 2 * s.cap ? 2 * s.cap : need;
    (void)hipFree(s.data);
    s.data = nullptr;
    s.cap = 0;
    if (hipMalloc((void**)&s.data, (size_t)want * sizeof(map_voxel_t)) != hipSuccess) {
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
  if (e == hipSuccess) e = gvom::launch_scan_i32(b->group_cnt, ng, b->n_occ + b->head, b->stream);
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
  if (e == hipSuccess)
    e = gvom::launch_fill_i32((int32_t*)m->occ, 0, (int64_t)m->p.nx * m->p.ny * d.W * 2,
                              b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->pushed, b->stream);
  if (e != hipSuccess) {
    m->sticky = MAP_E_DEVICE;
    return buf_fail(b, e);
  }
  m->empty = true;
  m->lut_counted = false;
  s.origin[0] = m->origin[0];
  s.origin[1] = m->origin[1];
  s.origin[2] = m->origin[2];
  b->head = (b->head + 1) % b->depth;
  if (b->count < b->depth) b->count++;
  return MAP_OK;
}

int32_t map_buffer_combine(map_buffer_t* b, map_t* out) {
  if (!b || !out) return MAP_E_INVALID;
  if (b->sticky) return b->sticky;
  if (out->sticky) return out->sticky;
  if (out->p.nx != b->p.nx || out->p.ny != b->p.ny || out->p.nz != b->p.nz ||
      out->p.res_m != b->p.res_m)
    return MAP_E_INVALID;
  if (b->count == 0) return MAP_E_INVALID;
  hipEvent_t ev = nullptr;
  if (!b->pool.empty()) {
    ev = b->pool.back();
    b->pool.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return MAP_E_DEVICE;
  }
  hipError_t e = hipStreamWaitEvent(out->stream, b->pushed, 0);
  const map_buffer_t::Slot& nw = b->slots[newest(b)];
  gvom::set_origin(out, nw.origin);
  out->lut_counted = false;
  out->empty = false;
  gvom::CombineArgs a;
  a.d = out->d;
  for (int i = 0; i < 3; i++) a.O[i] = nw.origin[i];
  a.k = b->count;
  for (int j = 0; j < b->count; j++) {
    const map_buffer_t::Slot& s = b->slots[(b->head + b->depth - b->count + j) % b->depth];
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
    hipLaunchKernelGGL(gvom::k_combine, dim3((unsigned)gvom::n_bricks(out->d)),
                       dim3(gvom::kBrickThreads), 0, out->stream, a);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev, out->stream);
  if (e != hipSuccess) {
    b->pool.push_back(ev);
    (void)hipGetLastError();
    out->sticky = MAP_E_DEVICE;
    return MAP_E_DEVICE;
  }
  b->pending.push_back(ev);
  return MAP_OK;
}

int32_t map_buffer_count(const map_buffer_t* b) { return b ? b->count : MAP_E_INVALID; }

int32_t map_buffer_get_stats(map_buffer_t* b, map_stats_t* out) {
  if (!b) return MAP_E_INVALID;
  return map_get_stats(b->prod, out);
}

}  // extern "C"
