// Host side of libgvom: the C ABI declared in include/gvom.h.  Validates
// arguments, owns the map state on the device, derives the host-side
// constants (sensor voxel, window origin, slabs to clear) and orders the
// kernel launches on the map's stream.  Nothing here waits on the device
// except where gvom.h says a call synchronises.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "gvom_internal.h"

using gvom::Dims;

struct map_t {
  map_params_t p;
  map_derived_t c;
  hipStream_t stream;
  int device;
  int32_t origin[3];
  Dims d;
  int32_t* hits;
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;
  int32_t* hq;
  int32_t* block_base;
  int32_t* colpre;
  unsigned long long* stats;  // 8 counters
  int32_t* err;
  uint32_t* touch;            // distinct-voxel bitmaps, allocated on first use
  int4* items;                // ray segments of the current insert
  int64_t item_cap;
  unsigned long long* part_rays;   // per-block counters of the ray pass
  unsigned long long* part_trace;  // per-block counters of the traversal pass
  int64_t part_rays_cap, part_trace_cap;
  int64_t last_ray_blocks, last_trace_blocks;
  int32_t seg_len;
  int32_t trace_wpc;
  int32_t n_cu;
  int32_t sticky;
  int64_t last_points, last_cleared;
  bool last_distinct;
  bool prof;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
};

namespace {

constexpr size_t kStatsBytes = (8 + gvom::kStripes) * 8;

int64_t n_vox(const map_t* m) { return (int64_t)m->p.nx * m->p.ny * m->p.nz; }
int64_t n_store(const map_t* m) { return m->d.vs; }
int64_t n_col(const map_t* m) { return (int64_t)m->p.nx * m->p.ny; }

int32_t pos_mod(int64_t a, int32_t n) {
  int64_t r = a % n;
  return (int32_t)(r < 0 ? r + n : r);
}

void set_ring(map_t* m) {
  m->d.ro[0] = pos_mod(m->origin[0], m->p.nx);
  m->d.ro[1] = pos_mod(m->origin[1], m->p.ny);
  m->d.ro[2] = pos_mod(m->origin[2], m->p.nz);
}

int32_t dev_status(map_t* m, hipError_t e) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    m->sticky = MAP_E_DEVICE;
    return MAP_E_DEVICE;
  }
  return MAP_OK;
}

// Enqueues: every voxel empty, every occupancy word zero.
hipError_t clear_all(map_t* m) {
  const int64_t V = n_store(m);
  hipError_t e = gvom::launch_fill_i32(m->hits, 0, V, m->stream);
  if (e == hipSuccess) e = gvom::launch_fill_i32(m->passes, 0, V, m->stream);
  if (e == hipSuccess) e = gvom::launch_fill_i32(m->minqz, INT32_MAX, V, m->stream);
  if (e == hipSuccess)
    e = gvom::launch_fill_i32((int32_t*)m->occ, 0, n_col(m) * m->d.W * 2, m->stream);
  return e;
}

void initial_origin(map_t* m) {
  m->origin[0] = -m->p.nx / 2;
  m->origin[1] = -m->p.ny / 2;
  m->origin[2] = -m->p.sensor_z_voxel;
  set_ring(m);
}

// Moves the window to new origin `o` (whole voxels, Sec. III-A): clears the
// storage slabs that the new window takes over from the old one.
hipError_t move_window(map_t* m, const int32_t o[3]) {
  const int32_t n[3] = {m->p.nx, m->p.ny, m->p.nz};
  int64_t delta[3];
  bool all = false;
  for (int a = 0; a < 3; a++) {
    delta[a] = (int64_t)o[a] - m->origin[a];
    if (delta[a] >= n[a] || -delta[a] >= n[a]) all = true;
  }
  m->last_cleared = 0;
  if (delta[0] == 0 && delta[1] == 0 && delta[2] == 0) return hipSuccess;
  for (int a = 0; a < 3; a++) m->origin[a] = o[a];
  set_ring(m);
  if (all) {
    m->last_cleared = n_vox(m);
    return clear_all(m);
  }
  int64_t keep = 1;
  for (int a = 0; a < 3; a++) keep *= n[a] - (delta[a] < 0 ? -delta[a] : delta[a]);
  m->last_cleared = n_vox(m) - keep;
  // storage range of the entering local range along axis a
  int32_t s0[3], cnt[3];
  for (int a = 0; a < 3; a++) {
    if (delta[a] > 0) {
      s0[a] = pos_mod((int64_t)n[a] - delta[a] + m->d.ro[a], n[a]);
      cnt[a] = (int32_t)delta[a];
    } else {
      s0[a] = m->d.ro[a];
      cnt[a] = (int32_t)-delta[a];
    }
  }
  hipError_t e = hipSuccess;
  if (cnt[0]) {
    e = gvom::launch_clear_box(m->d, m->hits, m->passes, m->minqz, s0[0], cnt[0], 0, n[1], 0,
                               n[2], m->stream);
    if (e == hipSuccess)
      e = gvom::launch_clear_occ(m->d, m->occ, s0[0], cnt[0], 0, n[1], 0ull, 0ull, m->stream);
  }
  if (cnt[1] && e == hipSuccess) {
    e = gvom::launch_clear_box(m->d, m->hits, m->passes, m->minqz, 0, n[0], s0[1], cnt[1], 0,
                               n[2], m->stream);
    if (e == hipSuccess)
      e = gvom::launch_clear_occ(m->d, m->occ, 0, n[0], s0[1], cnt[1], 0ull, 0ull, m->stream);
  }
  if (cnt[2] && e == hipSuccess) {
    e = gvom::launch_clear_box(m->d, m->hits, m->passes, m->minqz, 0, n[0], 0, n[1], s0[2],
                               cnt[2], m->stream);
    unsigned long long k0 = ~0ull, k1 = ~0ull;
    for (int j = 0; j < cnt[2]; j++) {
      const int z = (s0[2] + j) % n[2];
      if (z < 64) k0 &= ~(1ull << z); else k1 &= ~(1ull << (z - 64));
    }
    if (e == hipSuccess)
      e = gvom::launch_clear_occ(m->d, m->occ, 0, n[0], 0, n[1], k0, k1, m->stream);
  }
  return e;
}

// Records the start event of a profiled phase (no-op when profiling is off).
int prof_begin(map_t* m, int phase) {
  if (!m->prof) return -1;
  map_t::Mark k{phase, nullptr, nullptr};
  if (hipEventCreate(&k.a) != hipSuccess || hipEventCreate(&k.b) != hipSuccess) return -1;
  (void)hipEventRecord(k.a, m->stream);
  m->marks.push_back(k);
  return (int)m->marks.size() - 1;
}

void prof_end(map_t* m, int idx) {
  if (idx >= 0) (void)hipEventRecord(m->marks[idx].b, m->stream);
}

void prof_release(map_t* m) {
  for (auto& k : m->marks) {
    (void)hipEventDestroy(k.a);
    (void)hipEventDestroy(k.b);
  }
  m->marks.clear();
}

template <class T>
hipError_t dmalloc(T** p, size_t bytes) {
  return hipMalloc((void**)p, bytes < 16 ? 16 : bytes);
}

}  // namespace

extern "C" {

int32_t map_params_validate(const map_params_t* p, map_derived_t* out) {
  if (!p) return MAP_E_INVALID;
  if (p->nx < 2 || p->ny < 2 || p->nz < 1 || p->nx > 8192 || p->ny > 8192 || p->nz > 128)
    return MAP_E_INVALID;
  if ((p->nx & 1) || (p->ny & 1)) return MAP_E_INVALID;
  if ((int64_t)p->nx * p->ny * p->nz > 2147483647LL) return MAP_E_INVALID;
  if (!(p->res_m > 0.0f) || !isfinite(p->res_m)) return MAP_E_INVALID;
  if (p->sensor_z_voxel < 0 || p->sensor_z_voxel >= p->nz) return MAP_E_INVALID;
  if (!isfinite(p->obs_min_m) || !isfinite(p->obs_max_m) || p->obs_min_m < 0.0f ||
      p->obs_max_m < p->obs_min_m)
    return MAP_E_INVALID;
  if (p->dens_den <= 0 || p->dens_num < 0) return MAP_E_INVALID;
  if (p->fit_n < 3 || p->fit_n > 15 || !(p->fit_n & 1)) return MAP_E_INVALID;
  if (!isfinite(p->neg_thresh_m) || p->neg_thresh_m < 0.0f) return MAP_E_INVALID;
  if (!isfinite(p->neg_search_m) || p->neg_search_m < 0.0f) return MAP_E_INVALID;
  map_derived_t c;
  const double r = (double)p->res_m;
  c.inv_r = (float)(1.0 / r);
  const long lo = lround((double)p->obs_min_m / r);
  c.n_lo = (int32_t)(lo < 1 ? 1 : lo);
  c.n_hi = (int32_t)lround((double)p->obs_max_m / r);
  c.tau_neg_q = (int64_t)floor((double)p->neg_thresh_m / r * 65536.0);
  c.search_d = (int32_t)lround((double)p->neg_search_m / r);
  c.half_fit = (p->fit_n - 1) / 2;
  if (c.n_hi < c.n_lo) return MAP_E_INVALID;
  if (c.search_d < 1 || c.search_d > 64) return MAP_E_INVALID;
  if (out) *out = c;
  return MAP_OK;
}

int32_t map_create(const map_params_t* p, void* stream, map_t** out) {
  if (!out) return MAP_E_INVALID;
  *out = nullptr;
  map_derived_t c;
  int32_t s = map_params_validate(p, &c);
  if (s) return s;
  map_t* m = new (std::nothrow) map_t();
  if (!m) return MAP_E_OOM;
  m->p = *p;
  m->c = c;
  m->stream = (hipStream_t)stream;
  if (hipGetDevice(&m->device) != hipSuccess ||
      hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, m->device) !=
          hipSuccess) {
    delete m;
    return MAP_E_DEVICE;
  }
  m->seg_len = 32;
  m->trace_wpc = 32;
  m->part_trace_cap = (int64_t)m->n_cu * 32 / 4 + 1;
  m->d.nx = p->nx;
  m->d.ny = p->ny;
  m->d.nz = p->nz;
  m->d.W = (p->nz + 63) / 64;
  m->d.nby = (p->ny + 3) / 4;
  m->d.vs = (int64_t)((p->nx + 3) / 4) * m->d.nby * p->nz * 16;
  if (m->d.vs > 2147483647LL) {  // the 4-aligned storage must stay int32-indexable
    delete m;
    return MAP_E_INVALID;
  }
  const int64_t V = n_store(m), C = n_col(m);
  const int64_t nb = (C + 63) / 64;
  hipError_t e = dmalloc(&m->hits, V * 4);
  if (e == hipSuccess) e = dmalloc(&m->passes, V * 4);
  if (e == hipSuccess) e = dmalloc(&m->minqz, V * 4);
  if (e == hipSuccess) e = dmalloc(&m->occ, C * m->d.W * 8);
  if (e == hipSuccess) e = dmalloc(&m->hq, C * 4);
  if (e == hipSuccess) e = dmalloc(&m->block_base, nb * 4);
  if (e == hipSuccess) e = dmalloc(&m->colpre, C * 4);
  if (e == hipSuccess) e = dmalloc(&m->stats, kStatsBytes);
  if (e == hipSuccess) e = dmalloc(&m->err, 4);
  if (e == hipSuccess) e = dmalloc(&m->part_trace, m->part_trace_cap * 16);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    map_destroy(m);
    return MAP_E_OOM;
  }
  initial_origin(m);
  e = clear_all(m);
  if (e == hipSuccess) e = hipMemsetAsync(m->stats, 0, kStatsBytes, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    map_destroy(m);
    return MAP_E_DEVICE;
  }
  *out = m;
  return MAP_OK;
}

int32_t map_destroy(map_t* m) {
  if (!m) return MAP_OK;
  (void)hipStreamSynchronize(m->stream);
  prof_release(m);
  (void)hipFree(m->hits);
  (void)hipFree(m->passes);
  (void)hipFree(m->minqz);
  (void)hipFree(m->occ);
  (void)hipFree(m->hq);
  (void)hipFree(m->block_base);
  (void)hipFree(m->colpre);
  (void)hipFree(m->stats);
  (void)hipFree(m->err);
  (void)hipFree(m->touch);
  (void)hipFree(m->items);
  (void)hipFree(m->part_rays);
  (void)hipFree(m->part_trace);
  delete m;
  return MAP_OK;
}

int32_t map_reset(map_t* m) {
  if (!m) return MAP_E_INVALID;
  (void)hipStreamSynchronize(m->stream);
  (void)hipGetLastError();
  m->sticky = MAP_OK;
  initial_origin(m);
  m->last_points = 0;
  m->last_cleared = 0;
  m->last_distinct = false;
  m->last_ray_blocks = 0;
  m->last_trace_blocks = 0;
  hipError_t e = clear_all(m);
  if (e == hipSuccess) e = hipMemsetAsync(m->stats, 0, kStatsBytes, m->stream);
  return dev_status(m, e);
}

int32_t map_insert_scan(map_t* m, const float* xyz_dev, int64_t n, const float pose[12],
                        uint32_t flags) {
  if (!m || !pose || n < 0 || n > 2147483647LL || (n > 0 && !xyz_dev)) return MAP_E_INVALID;
  if (flags & 0x0000FFFCu) return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  for (int i = 0; i < 12; i++)
    if (!isfinite(pose[i])) return MAP_E_POSE;
  int32_t S[3], sv[3];
  for (int i = 0; i < 3; i++) {
    const float u = pose[4 * i + 3] * m->c.inv_r;
    if (!(fabsf(u) < 32768.0f)) return MAP_E_RANGE;
    S[i] = (int32_t)floorf(u * 65536.0f);
    sv[i] = S[i] >> 16;
  }
  // segment buffer for the traversal pass (grows before any work is enqueued):
  // ray block b writes into the region of stripe b mod kStripes, sized for the
  // most segments that stripe's points can produce
  const int64_t ray_blocks = (n + gvom::kRayBlock - 1) / gvom::kRayBlock;
  const int64_t per_ray = gvom::max_segments(m->d, m->seg_len);
  int64_t stripe_off[gvom::kStripes], stripe_cap[gvom::kStripes], need = 0;
  for (int t = 0; t < gvom::kStripes; t++) {
    const int64_t blocks = ray_blocks > t ? (ray_blocks - t + gvom::kStripes - 1) / gvom::kStripes : 0;
    int64_t pts = blocks * gvom::kRayBlock;
    if (blocks && t == (ray_blocks - 1) % gvom::kStripes)
      pts -= ray_blocks * gvom::kRayBlock - n;  // the last block is partial
    stripe_off[t] = need;
    stripe_cap[t] = pts * per_ray;
    need += stripe_cap[t];
  }
  if (need > m->item_cap) {
    if (hipStreamSynchronize(m->stream) != hipSuccess) return dev_status(m, hipErrorUnknown);
    (void)hipFree(m->items);
    m->items = nullptr;
    m->item_cap = 0;
    if (dmalloc(&m->items, (size_t)need * sizeof(int4)) != hipSuccess) {
      (void)hipGetLastError();
      m->items = nullptr;
      return MAP_E_OOM;
    }
    m->item_cap = need;
  }
  if (ray_blocks > m->part_rays_cap) {
    if (hipStreamSynchronize(m->stream) != hipSuccess) return dev_status(m, hipErrorUnknown);
    (void)hipFree(m->part_rays);
    m->part_rays = nullptr;
    m->part_rays_cap = 0;
    if (dmalloc(&m->part_rays, (size_t)ray_blocks * 32) != hipSuccess) {
      (void)hipGetLastError();
      m->part_rays = nullptr;
      return MAP_E_OOM;
    }
    m->part_rays_cap = ray_blocks;
  }
  hipError_t e = hipSuccess;
  if (flags & MAP_RECENTER) {
    const int32_t o[3] = {sv[0] - m->p.nx / 2, sv[1] - m->p.ny / 2,
                          sv[2] - m->p.sensor_z_voxel};
    const int pm = prof_begin(m, MAP_PROF_SCROLL);
    e = move_window(m, o);
    prof_end(m, pm);
  } else {
    const int32_t n3[3] = {m->p.nx, m->p.ny, m->p.nz};
    for (int a = 0; a < 3; a++) {
      const int64_t l = (int64_t)sv[a] - m->origin[a];
      if (l < 0 || l >= n3[a]) return MAP_E_SENSOR_OUTSIDE;
    }
    m->last_cleared = 0;
  }
  const bool distinct = (flags & MAP_STATS_DISTINCT) != 0;
  m->last_points = n;
  m->last_distinct = distinct;
  m->last_ray_blocks = 0;
  m->last_trace_blocks = 0;
  if (e == hipSuccess) e = hipMemsetAsync(m->stats, 0, kStatsBytes, m->stream);
  if (distinct && e == hipSuccess) {
    const int64_t words = (n_store(m) + 31) / 32;
    if (!m->touch) e = dmalloc(&m->touch, words * 2 * 4);
    if (e == hipSuccess) e = hipMemsetAsync(m->touch, 0, words * 2 * 4, m->stream);
  }
  if (e == hipSuccess && n > 0) {
    gvom::InsertArgs a;
    a.xyz = xyz_dev;
    a.n = (int32_t)n;
    uint32_t fw = flags >> 16;
    if (fw < 1 || n % fw != 0) fw = 1;
    a.fw = (int32_t)fw;
    a.azimuths = (int32_t)(n / fw);
    for (int i = 0; i < 3; i++) {
      for (int j = 0; j < 3; j++) a.R[3 * i + j] = pose[4 * i + j];
      a.t[i] = pose[4 * i + 3];
      a.S[i] = S[i];
      a.O[i] = m->origin[i];
    }
    a.inv_r = m->c.inv_r;
    a.d = m->d;
    a.hits = m->hits;
    a.passes = m->passes;
    a.minqz = m->minqz;
    a.occ = m->occ;
    a.stats = m->stats;
    a.touch = m->touch;
    a.items = m->items;
    for (int t = 0; t < gvom::kStripes; t++) {
      a.stripe_off[t] = stripe_off[t];
      a.stripe_cap[t] = stripe_cap[t];
    }
    a.part_rays = m->part_rays;
    a.part_trace = m->part_trace;
    a.item_cap = m->item_cap;
    a.seg_len = m->seg_len;
    {
      const int64_t want = (need + 255) / 256;
      const int64_t lim = (int64_t)m->n_cu * m->trace_wpc / 4;
      a.trace_blocks = (int32_t)(want < lim ? want : lim);
    }
    m->last_ray_blocks = ray_blocks;
    m->last_trace_blocks = a.trace_blocks;
    const int pm = prof_begin(m, MAP_PROF_INSERT);
    e = gvom::launch_insert(a, distinct, m->stream);
    prof_end(m, pm);
  }
  return dev_status(m, e);
}

int32_t map_export_2d(map_t* m, const map_2d_t* out) {
  if (!m || !out || !out->height || !out->slope || !out->rough || !out->density || !out->flags)
    return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  gvom::ColumnArgs ca;
  ca.d = m->d;
  ca.hits = m->hits;
  ca.passes = m->passes;
  ca.minqz = m->minqz;
  ca.occ = m->occ;
  ca.res = (double)m->p.res_m;
  ca.n_lo = m->c.n_lo;
  ca.n_hi = m->c.n_hi;
  ca.dens_num = m->p.dens_num;
  ca.dens_den = m->p.dens_den;
  ca.height = out->height;
  ca.density = out->density;
  ca.flags = out->flags;
  ca.hq = m->hq;
  int pm = prof_begin(m, MAP_PROF_COLUMN);
  hipError_t e = gvom::launch_column(ca, m->stream);
  prof_end(m, pm);
  if (e == hipSuccess) {
    gvom::SurfaceArgs sa;
    sa.nx = m->p.nx;
    sa.ny = m->p.ny;
    sa.hq = m->hq;
    sa.half_fit = m->c.half_fit;
    sa.search_d = m->c.search_d;
    sa.tau_q = m->c.tau_neg_q;
    sa.q2m = (double)m->p.res_m / 65536.0;
    sa.slope = out->slope;
    sa.rough = out->rough;
    sa.flags = out->flags;
    pm = prof_begin(m, MAP_PROF_SURFACE);
    e = gvom::launch_surface(sa, m->stream);
    prof_end(m, pm);
  }
  return dev_status(m, e);
}

int32_t map_export_voxels(map_t* m, int32_t* lut_dev, map_voxel_t* data_dev, int64_t cap,
                          int64_t* n_occupied_dev, int32_t origin_vox[3]) {
  if (!m || !lut_dev || !n_occupied_dev || !origin_vox || cap < 0 || (cap > 0 && !data_dev))
    return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  gvom::LutArgs a;
  a.d = m->d;
  a.hits = m->hits;
  a.passes = m->passes;
  a.minqz = m->minqz;
  a.occ = m->occ;
  a.lut = lut_dev;
  a.data = data_dev;
  a.cap = cap;
  a.block_base = m->block_base;
  a.colpre = m->colpre;
  a.n_occupied = n_occupied_dev;
  const int pm = prof_begin(m, MAP_PROF_LUT);
  hipError_t e = gvom::launch_lut(a, m->stream);
  prof_end(m, pm);
  for (int i = 0; i < 3; i++) origin_vox[i] = m->origin[i];
  return dev_status(m, e);
}

int32_t map_import_voxels(map_t* m, const int32_t* lut_dev, const map_voxel_t* data_dev,
                          int64_t n_data, const int32_t origin_vox[3]) {
  if (!m || !lut_dev || !origin_vox || n_data < 0 || (n_data > 0 && !data_dev))
    return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  for (int i = 0; i < 3; i++) m->origin[i] = origin_vox[i];
  set_ring(m);
  int32_t err = 0;
  hipError_t e = hipMemsetAsync(m->err, 0, 4, m->stream);
  if (e == hipSuccess)
    e = gvom::launch_import(m->d, lut_dev, data_dev, n_data, m->hits, m->passes, m->minqz,
                            m->occ, m->err, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&err, m->err, 4, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return dev_status(m, e);
  if (err) {
    initial_origin(m);
    e = clear_all(m);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return dev_status(m, e);
    return MAP_E_INVALID;
  }
  return MAP_OK;
}

int32_t map_get_stats(map_t* m, map_stats_t* out) {
  if (!m || !out) return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  std::vector<unsigned long long> pr((size_t)m->last_ray_blocks * 4 + 1),
      pt((size_t)m->last_trace_blocks * 2 + 1);
  hipError_t e = hipSuccess;
  if (m->last_ray_blocks)
    e = hipMemcpyAsync(pr.data(), m->part_rays, m->last_ray_blocks * 32, hipMemcpyDeviceToHost,
                       m->stream);
  if (e == hipSuccess && m->last_trace_blocks)
    e = hipMemcpyAsync(pt.data(), m->part_trace, m->last_trace_blocks * 16,
                       hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return dev_status(m, e);
  int64_t c[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t b = 0; b < m->last_ray_blocks; b++) {
    c[0] += (int64_t)pr[4 * b + 0];
    c[1] += (int64_t)pr[4 * b + 1];
    c[2] += (int64_t)pr[4 * b + 2];
    c[5] += (int64_t)pr[4 * b + 3];
  }
  for (int64_t b = 0; b < m->last_trace_blocks; b++) {
    c[3] += (int64_t)pt[2 * b + 0];
    c[4] += (int64_t)pt[2 * b + 1];
  }
  out->n_points = m->last_points;
  out->n_nonfinite = c[0];
  out->n_range = c[1];
  out->n_hits = c[2];
  out->n_pass = c[3];
  out->n_distinct_pass = m->last_distinct ? c[4] : -1;
  out->n_distinct_hit = m->last_distinct ? c[5] : -1;
  out->n_cleared = m->last_cleared;
  return MAP_OK;
}

int32_t map_get_origin(const map_t* m, int32_t origin_vox[3]) {
  if (!m || !origin_vox) return MAP_E_INVALID;
  for (int i = 0; i < 3; i++) origin_vox[i] = m->origin[i];
  return MAP_OK;
}

int32_t map_sync(map_t* m) {
  if (!m) return MAP_E_INVALID;
  if (m->sticky) return m->sticky;
  return dev_status(m, hipStreamSynchronize(m->stream));
}

int32_t map_set_tuning(map_t* m, const map_tuning_t* t) {
  if (!m || !t) return MAP_E_INVALID;
  if (t->seg_len > 1024 || t->trace_waves_per_cu > 32) return MAP_E_INVALID;
  if (t->seg_len > 0 && t->seg_len != m->seg_len) {
    // the segment buffer is sized for the segment length: regrow on next insert
    if (hipStreamSynchronize(m->stream) != hipSuccess) return dev_status(m, hipErrorUnknown);
    (void)hipFree(m->items);
    m->items = nullptr;
    m->item_cap = 0;
    m->seg_len = t->seg_len;
  }
  if (t->trace_waves_per_cu > 0) m->trace_wpc = t->trace_waves_per_cu;
  return MAP_OK;
}

int32_t map_get_tuning(const map_t* m, map_tuning_t* out) {
  if (!m || !out) return MAP_E_INVALID;
  out->seg_len = m->seg_len;
  out->trace_waves_per_cu = m->trace_wpc;
  return MAP_OK;
}

int32_t map_profile_enable(map_t* m, int32_t enable) {
  if (!m) return MAP_E_INVALID;
  m->prof = enable != 0;
  return MAP_OK;
}

int32_t map_profile_read(map_t* m, double ms[MAP_PROF_N], int64_t count[MAP_PROF_N]) {
  if (!m || !ms || !count) return MAP_E_INVALID;
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return dev_status(m, e);
  for (auto& k : m->marks) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, k.a, k.b) == hipSuccess) {
      ms[k.phase] += t;
      count[k.phase] += 1;
    }
  }
  prof_release(m);
  return MAP_OK;
}

const char* map_status_str(int32_t s) {
  switch (s) {
    case MAP_OK: return "ok";
    case MAP_E_INVALID: return "invalid argument";
    case MAP_E_POSE: return "non-finite pose";
    case MAP_E_SENSOR_OUTSIDE: return "sensor outside the map window";
    case MAP_E_RANGE: return "sensor position out of range";
    case MAP_E_CAPACITY: return "output buffer too small";
    case MAP_E_OOM: return "device allocation failed";
    case MAP_E_DEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

}  // extern "C"
