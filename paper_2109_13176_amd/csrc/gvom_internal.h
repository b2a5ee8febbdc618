// Internal declarations shared by the host code and the kernels of libgvom.
//
// Storage layout on the device (per map):
//   hits, passes, min_qz : int32 per voxel, TOROIDAL: world voxel g is stored
//                          at storage coordinate s = (g mod nx, g mod ny,
//                          g mod nz), so a moving window only clears the slabs
//                          it enters.  Columns are grouped in 4 x 4 bricks:
//                          voxel s lives at col_base(sx, sy) + 16 sz, so one
//                          64-byte line holds one z level of a brick and
//                          neighbouring columns share lines.
//   occ                  : uint64[nx*ny][W], W = ceil(nz/64): bit (s mod 64) of
//                          word s/64 is set iff storage z = s of that column
//                          holds a return (hits >= 1).
// "ro" is the ring offset origin mod n per axis: window-local coordinate l
// is stored at (l + ro) mod n.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gvom.h"

namespace gvom {

// Device allocations of the library go through these two calls, which keep
// the process-wide total that map_set_device_memory_limit caps.
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t dev_free(void* p);

struct Dims {
  int32_t nx, ny, nz, W;  // W = occupancy words per column
  int32_t ro[3];          // ring offsets
  int32_t nby;            // bricks along y = ceil(ny / 4)
  int64_t vs;             // storage voxels = ceil(nx/4) * nby * nz * 16
};

// Storage index of z = 0 of storage column (sx, sy); z adds 16 per level.
__host__ __device__ __forceinline__ int32_t col_base(const Dims& d, int32_t sx, int32_t sy) {
  return ((((sx >> 2) * d.nby + (sy >> 2)) * d.nz) << 4) + ((sy & 3) << 2) + (sx & 3);
}

constexpr int kStripes = 16;  // independent segment counters of the ray pass
static_assert((kStripes & (kStripes - 1)) == 0, "the traversal binary-searches the stripes");

// Sensor box of the segmented traversal: every ray starts in the sensor's
// voxel, so the cells around it take the passes of thousands of waves and
// device atomics on their few cache lines serialize.  Passes of cells inside a
// kBoxXY x kBoxXY x kBoxZ box around the sensor are summed per block in LDS,
// flushed into one of kBoxReps replicas of the box, and the replicas are
// added into the map by a small fold kernel.
constexpr int kBoxXY = 17;
constexpr int kBoxZ = 9;
constexpr int kBoxCells = kBoxXY * kBoxXY * kBoxZ;
constexpr int kBoxReps = 128;

struct InsertArgs {
  const float* xyz;
  int32_t n;
  int32_t fw;             // firing width (1 = identity order)
  int32_t azimuths;       // n / fw
  float R[9], t[3];
  float inv_r;
  int32_t S[3];           // sensor, Q units
  int32_t O[3];           // window origin, world voxel
  Dims d;
  int32_t* hits;
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;
  unsigned long long* stats;   // [8 global counters][kStripes segment counters]
  uint32_t* touch;             // distinct-voxel bitmaps [2][V/32] or null
  unsigned long long* part_rays;   // per ray block: nonfinite, range, hits, distinct hits
  unsigned long long* part_trace;  // per trace block: passes, distinct passes, updates, 0
  int4* rays;                  // per ray (ray-pass lane): {Qx, Qy, Qz, segments}
  int2* witems;                // wave items {ray wave, segment index}, per stripe
  int64_t stripe_off[kStripes];  // wave-item region of each stripe of ray blocks
  int64_t stripe_cap[kStripes];
  int32_t seg_len;             // dominant-axis voxels per segment
  int32_t trace_blocks;        // grid of the trace kernel (kTraceBlock threads per block
                               // for a single map, 256 in a batch)
  // sensor box (segmented traversal): storage coordinate of its first cell
  // and extent per axis; cell (dx, dy, dz) has box index
  // (dx * kBoxXY + dy) * kBoxZ + dz
  int32_t box_s[3];
  int32_t box_e[3];
  int32_t box_l[3];            // window-local coordinate of the box's first cell
  int32_t* box_rep;            // [kBoxReps][kBoxCells], zero between inserts
};

constexpr int kBlock = 256;       // threads per block of the plain kernels
constexpr int kRayBlock = 512;    // threads per block of the ray pass (rays regrouped per block)
// threads per block of the traversal (single map and batch): four waves
// share one LDS copy of the sensor box; small blocks let seven of them fit a
// CU (LDS and registers), and the walk is bound by per-wave latency
constexpr int kTraceBlock = 256;
constexpr int kTraceWavesPerSimd = 7;

// Blocks of the sensor-box fold that follows the segmented traversal.
int box_fold_blocks();
// Replica groups of the fold (each fold block sums one group of replicas).
int box_fold_groups();

// Segments one ray can produce at most.
int64_t max_segments(const Dims& d, int32_t seg_len);

struct ColumnArgs {
  Dims d;
  const int32_t* hits;
  const int32_t* passes;
  const int32_t* minqz;
  const unsigned long long* occ;
  double res;
  int32_t n_lo, n_hi;
  int32_t dens_num, dens_den;
  float* height;
  float* density;
  uint8_t* flags;
  int32_t* hq;            // ground height Q per local pixel, INT32_MIN = undefined
  int32_t* colpre;        // null, or the table export's counting pass (see LutArgs)
  int32_t* block_base;
};

struct SurfaceArgs {
  int32_t nx, ny;
  const int32_t* hq;
  int32_t half_fit;
  int32_t search_d;
  int64_t tau_q;
  double q2m;             // metres per Q unit = res / 65536
  float* slope;
  float* rough;
  uint8_t* flags;
};

struct LutArgs {
  Dims d;
  const int32_t* hits;
  const int32_t* passes;
  const int32_t* minqz;
  const unsigned long long* occ;
  int32_t* lut;
  map_voxel_t* data;
  int64_t cap;
  int32_t* block_base;    // per group of 64 window-local columns: exclusive rank base
  int32_t* colpre;        // per window-local column: exclusive rank within its group
  int64_t* n_occupied;
};

struct DensityArgs {
  Dims d;
  const int32_t* hits;
  const int32_t* passes;
  float* out;             // [nx*ny*nz], window-local table order
};

struct CostArgs {
  int64_t n;              // pixels
  const float* slope;
  const float* rough;
  const float* density;
  const uint8_t* flags;
  float w[8];             // slope, rough, density, positive, hard, soft, negative, unknown
  float* cost;
};

struct ClearArgs {
  Dims d;
  int32_t* hits;
  int32_t* passes;
  int32_t* minqz;
  unsigned long long* occ;
  int32_t nbox;
  int32_t box[3][6];              // x0, cx, y0, cy, z0, cz (storage coordinates)
  unsigned long long keep[3][2];  // occupancy bits kept in the box's columns
};

// ---- batches of maps ------------------------------------------------------
constexpr int kMaxBatch = 64;

// Per-step table of a batch: virtual-block prefixes of every stage (block b of
// stage S belongs to the map m with pre[m] <= b < pre[m+1]) and per-map
// launch constants.  Lives in device memory, uploaded once per step.  The
// surface pass has one prefix per tile size (index 0: 16, 1: 32); a map has
// blocks only in the prefix of its own tile.
struct BatchStep {
  int32_t nmaps;
  int32_t pre_rays[kMaxBatch + 1];
  int32_t pre_trace[kMaxBatch + 1];
  int32_t pre_col[kMaxBatch + 1];
  int32_t pre_surf[2][kMaxBatch + 1];
  int32_t pre_lcount[kMaxBatch + 1];
  int32_t pre_lscan[kMaxBatch + 1];
  int32_t pre_lwrite[kMaxBatch + 1];
  int32_t surf_tiles_y[kMaxBatch];
  int32_t surf_H[kMaxBatch];
  int32_t lw_by[kMaxBatch];
  int32_t lut_groups[kMaxBatch];
  uint32_t nz_magic[kMaxBatch];
  int32_t last_is_lut[kMaxBatch];
};

struct BatchTables {
  BatchStep st;
  ClearArgs clr[kMaxBatch];
  InsertArgs ins[kMaxBatch];
  ColumnArgs col[kMaxBatch];
  SurfaceArgs sur[kMaxBatch];
  LutArgs lut[kMaxBatch];
};

struct BatchGrid {
  int clear, rays, trace, col, surf, surf16, lcount, lwrite;  // persistent grid sizes
  int fold;                                                   // maps x sensor-box fold blocks
  size_t surf_lds, lut_lds;
};

// Enqueues one batched step (all stages of all maps) reading `tab` (device).
// stamps[0] = step start, stamps[1 + m] = completion of map m (wall clock:
// the latest end of its last-stage blocks).
hipError_t launch_batch_insert(const BatchTables* tab, const BatchGrid& g,
                               unsigned long long* stamps, hipStream_t s);
hipError_t launch_batch_export(const BatchTables* tab, const BatchGrid& g,
                               unsigned long long* stamps, hipStream_t s);
int surface_tile();
size_t surface_lds(int H, int tile);
size_t lut_lds(int nz);
uint32_t nz_magic(int nz);

// Launchers (all enqueue on `s`, return the launch status).
hipError_t launch_clear(const ClearArgs& a, hipStream_t s);
hipError_t launch_rays(const InsertArgs& a, bool distinct, hipStream_t s);
hipError_t launch_trace(const InsertArgs& a, bool distinct, hipStream_t s);
hipError_t launch_column(const ColumnArgs& a, hipStream_t s);
hipError_t launch_surface(const SurfaceArgs& a, int tile, hipStream_t s);  // tile 16 or 32
// counted: the column pass already wrote colpre / block_base for this state
hipError_t launch_lut(const LutArgs& a, bool counted, hipStream_t s);
hipError_t launch_import(const Dims& d, const int32_t* lut, const map_voxel_t* data,
                         int64_t n_data, int32_t* hits, int32_t* passes, int32_t* minqz,
                         unsigned long long* occ, int32_t* err, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// out[0..3] = column sums of the ray pass's per-block counters parts[nblocks][4].
hipError_t launch_sum_ray_parts(const unsigned long long* parts, int64_t nblocks,
                                unsigned long long* out, hipStream_t s);
hipError_t launch_density(const DensityArgs& a, hipStream_t s);
hipError_t launch_costmap(const CostArgs& a, hipStream_t s);
// Exclusive prefix of base[0..nb) in place (one block); *total = the sum.
hipError_t launch_scan_i32(int32_t* base, int nb, int64_t* total, hipStream_t s);

}  // namespace gvom
