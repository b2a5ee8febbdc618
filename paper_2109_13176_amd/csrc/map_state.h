// Host-side state of one map (shared by the host sources of libgvom).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "gvom_internal.h"

struct map_t {
  map_params_t p;
  map_derived_t c;
  hipStream_t stream;
  int device;
  int32_t origin[3];
  gvom::Dims d;
  int32_t* hits;
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;
  int32_t* hq;
  int32_t* block_base;
  int32_t* colpre;
  unsigned long long* stats;  // 8 counters
  int32_t* err;
  int64_t* nocc;              // occupied-voxel count of a synchronous table export
  uint32_t* touch;            // distinct-voxel bitmaps, allocated on first use
  int4* rays;                 // per-ray records of the current insert
  int2* witems;               // its wave items
  int64_t rays_cap, witem_cap;
  unsigned long long* part_rays;   // per-block counters of the ray pass
  unsigned long long* part_trace;  // per-block counters of the traversal pass
  int64_t part_rays_cap, part_trace_cap;
  int64_t last_ray_blocks, last_trace_blocks;
  int32_t seg_len;
  int32_t trace_wpc;
  int32_t surf_tile;           // 16 or 32
  int32_t* box_rep;           // sensor-box replicas of the segmented traversal
  int32_t n_cu;
  int32_t sticky;
  int64_t last_points, last_cleared;
  bool last_distinct;
  // the last insert ran from the device's static scratch: its ray-pass
  // counters were summed into stats[0..3] (the per-block ones are not kept)
  bool last_static;
  int32_t prof_mask;          // profiled phases (bit p = phase p)
  // the last 2D export left the table export's per-column ranks (colpre,
  // block_base) for the current map state; any change of the map clears it
  bool lut_counted;
  // every voxel is empty and every occupancy word zero (a recentring then
  // needs no clears)
  bool empty;
  // a fresh value (from a process-wide counter) whenever the voxel state may
  // change: a combine can tell that a map still holds its previous result
  uint64_t version;
  struct Mark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
};

namespace gvom {
// Sets the window origin (whole voxels) and its ring offsets; the voxel state
// is not touched.
void set_origin(map_t* m, const int32_t o[3]);
// Same, for a map whose state is empty (no clears are needed).
void set_empty_origin(map_t* m, const int32_t o[3]);
// Next value of the process-wide state version counter (never 0).
uint64_t next_version();
}  // namespace gvom

