/*
 * gvom.h -- C ABI of the MI355X per-scan voxel-mapping library (libgvom.so).
 *
 * The library implements the per-scan path of G-VOM (Overbye & Saripalli,
 * "G-VOM: A GPU Accelerated Voxel Off-Road Mapping System", arXiv 2109.13176):
 * a lidar scan and its odometry pose go in (Sec. I: the system needs only
 * odometry and lidar); the points are transformed into the map frame and
 * binned into a robot-centred voxel map whose voxels carry hits, passes and
 * the lowest return height (Sec. III-A, III-C); the map is exported as the
 * lookup table + data array of Sec. III-A and as the 2D height, obstacle,
 * slope, roughness and negative-obstacle maps of Sec. III-D.
 *
 * Conventions for every call:
 *  - Every call returns an int32_t status: MAP_OK (0) or a negative MAP_E_*.
 *    Nothing throws or aborts across the ABI.
 *  - Bulk buffers (points, outputs) are DEVICE pointers owned by the caller.
 *    Poses, parameters and small results are HOST pointers.  The library owns
 *    only the map state it allocates in map_create.
 *  - Work is enqueued on the map's HIP stream (hipStream_t passed as void*;
 *    NULL = the default stream) and the call returns without waiting, except
 *    where a call says it synchronises.  Outputs are valid once that stream
 *    has been synchronised.
 *  - An error detected before any work is enqueued leaves the map unchanged.
 *    A HIP runtime error marks the map with the sticky MAP_E_DEVICE, which
 *    every later call returns until map_reset.
 *  - Different maps may be used from different threads; one map is not
 *    thread-safe.
 *
 * Coordinates.  World coordinates are metres.  A "Q" value is a coordinate in
 * units of 2^-16 voxel edge (int32); the voxel of a Q value is floor(Q/2^16).
 * The window holds nx*ny*nz voxels; its origin (world voxel index of window
 * voxel (0,0,0)) is always a whole number of voxels (Sec. III-A).  Window-local
 * voxel (x, y, z) has linear index (x*ny + y)*nz + z; 2D maps are [nx][ny]
 * with y fastest.
 */
#ifndef GVOM_H
#define GVOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MAP_OK                 0
#define MAP_E_INVALID         -1  /* null pointer, n < 0, bad parameter or flag      */
#define MAP_E_POSE            -2  /* non-finite pose                                 */
#define MAP_E_SENSOR_OUTSIDE  -3  /* sensor voxel outside the window, no recentring  */
#define MAP_E_RANGE           -4  /* sensor |t / res| >= 2^15 voxels                 */
#define MAP_E_CAPACITY        -5  /* an output buffer is too small                   */
#define MAP_E_OOM             -6  /* device allocation failed                        */
#define MAP_E_DEVICE          -7  /* HIP runtime error (sticky until map_reset)      */

/* ---- map_insert_scan flags -------------------------------------------- */
#define MAP_RECENTER        1u   /* move the window onto the pose before inserting   */
#define MAP_STATS_DISTINCT  2u   /* also count distinct voxels touched (slower)      */
/* Performance hint only (results never depend on it): the cloud is ordered
 * as consecutive firings of b beams (point index = azimuth * b + beam), as a
 * spinning lidar delivers it.  b in [1, 65535]. */
#define MAP_FIRING(b)       (((uint32_t)(b) & 0xFFFFu) << 16)

/* ---- parameters -------------------------------------------------------- */
/* The paper names every parameter below but fixes none of their values. */
typedef struct {
  int32_t nx, ny, nz;       /* window size in voxels; nx, ny even in [2, 8192]; nz in
                               [1, 128]; nx*ny*nz < 2^31 (Sec. III-A)                 */
  float   res_m;            /* cubic voxel edge in metres, > 0 (Sec. III-A)          */
  int32_t sensor_z_voxel;   /* window z index of the sensor voxel after recentring   */
  float   obs_min_m;        /* positive-obstacle band above the ground voxel,        */
  float   obs_max_m;        /*   min and max height (Sec. III-D)                      */
  int32_t dens_num;         /* hard obstacle iff band density > dens_num / dens_den  */
  int32_t dens_den;         /*   (Sec. III-D); dens_den > 0, dens_num >= 0            */
  int32_t fit_n;            /* odd N of the N x N plane fit, 3..15 (Sec. III-D)       */
  float   neg_thresh_m;     /* negative-obstacle height-difference threshold         */
  float   neg_search_m;     /* maximum cone-search distance (Sec. III-D)             */
} map_params_t;

/* Integer constants the library derives from the parameters (host only).
 * Rounding is half away from zero, computed in double. */
typedef struct {
  float   inv_r;            /* (float)(1 / (double)res_m)                             */
  int32_t n_lo, n_hi;       /* band in voxels above ground: max(1, round(min/r)),
                               round(max/r)                                           */
  int64_t tau_neg_q;        /* floor(neg_thresh / r * 2^16), in Q units              */
  int32_t search_d;         /* round(neg_search / r) pixels, 1..64                    */
  int32_t half_fit;         /* (fit_n - 1) / 2                                        */
} map_derived_t;

/* Outputs of map_export_2d: device arrays of nx*ny elements ([x][y], y fastest).
 * flags: bit0 height defined, bit1 positive obstacle, bit2 hard, bit3 soft,
 * bit4 negative obstacle, bit5 slope/roughness defined.  Undefined floats are
 * the quiet NaN 0x7FC00000. */
typedef struct {
  float*   height;    /* m: lowest return of the lowest occupied voxel            */
  float*   slope;     /* rise over run of the N x N least-squares plane           */
  float*   rough;     /* m^2: mean squared residual of that plane                 */
  float*   density;   /* sum hits / sum (hits + passes) over the obstacle band    */
  uint8_t* flags;
} map_2d_t;

/* One entry of the data array (Sec. III-A): returns in the voxel, rays that
 * passed through it, and the lowest return height in Q units. */
typedef struct {
  int32_t hits, passes, min_qz;
} map_voxel_t;

/* Counters of the last map_insert_scan (map_get_stats synchronises). */
typedef struct {
  int64_t n_points;         /* points given, including non-finite ones            */
  int64_t n_nonfinite;      /* skipped: a coordinate is NaN or infinite            */
  int64_t n_range;          /* skipped: |u| >= 2^15 voxels or >= 2048 voxels from
                               the sensor on an axis                               */
  int64_t n_hits;           /* returns whose voxel lies in the window             */
  int64_t n_pass;           /* pass increments (ray-voxel incidences)             */
  int64_t n_distinct_pass;  /* distinct voxels passed (-1 without MAP_STATS_DISTINCT) */
  int64_t n_distinct_hit;   /* distinct voxels hit   (-1 without MAP_STATS_DISTINCT) */
  int64_t n_cleared;        /* window voxels reset by the recentring              */
  int64_t n_pass_updates;   /* global-memory pass updates the traversal issued,
                               not counting the cells next to the sensor, which
                               are summed on chip first (diagnostic: depends on
                               the work order, so it is not reproducible from run
                               to run)                                            */
} map_stats_t;

typedef struct map_t map_t;  /* opaque */

/* Caps the device memory this library allocates in the process (the state of
 * every map, buffer, batch and network, and their per-scan work buffers) at
 * `bytes`; 0 removes the cap.  An allocation that would exceed the cap fails
 * as if the device were out of memory, so the call that needed it returns
 * MAP_E_OOM (a map_insert_scan that cannot grow its work buffers leaves the
 * map unchanged).  Memory already held is not affected.  MAP_E_INVALID for
 * bytes < 0.  For processes that share the GPU with other work. */
int32_t map_set_device_memory_limit(int64_t bytes);
/* Device memory, in bytes, the library holds in this process. */
int64_t map_device_memory_in_use(void);

/* Checks the parameters and derives the integer constants; host only, no HIP
 * call.  Returns MAP_E_INVALID for any parameter outside the ranges above. */
int32_t map_params_validate(const map_params_t* p, map_derived_t* out);

/* Creates an empty map (Sec. III-A storage) on the current HIP device, bound
 * to `stream`.  Until the first recentring the window is placed so that world
 * point (0,0,0) lies in voxel (nx/2, ny/2, sensor_z_voxel).  Allocates about
 * 12 bytes per voxel plus 16 bytes per column.  Synchronises. */
int32_t map_create(const map_params_t* p, void* stream, map_t** out);

/* Frees the map (synchronises its stream first).  NULL is a no-op. */
int32_t map_destroy(map_t* m);

/* Empties the map, restores the initial window and clears a sticky error. */
int32_t map_reset(map_t* m);

/* Inserts one lidar scan (Sec. III-C).
 *  xyz_dev: device float[n][3], sensor frame, metres; non-finite = no return
 *           (skipped, counted).  Not modified; must stay valid until the
 *           stream reaches this work.
 *  pose:    host float[12], row-major [R | t], sensor to world.
 *  flags:   MAP_RECENTER, MAP_STATS_DISTINCT, MAP_FIRING(b).
 * Each point is transformed with one fused multiply-add chain per axis
 * (t + R0 x + R1 y + R2 z, binary32), scaled to voxel units and quantised to
 * Q.  Its voxel, if in the window, gets hits += 1 and min_qz = min(min_qz, Qz);
 * every other window voxel on the segment from the sensor to the point gets
 * passes += 1 (the voxels of the segment are the distinct cells floor(X(t))
 * in increasing t; a boundary belongs to the upper cell).  n == 0 is allowed;
 * the recentring still happens.  Several lidars feed one map by calling this
 * once per lidar (Sec. III-B). */
int32_t map_insert_scan(map_t* m, const float* xyz_dev, int64_t n, const float pose[12],
                        uint32_t flags);

/* map_insert_scan for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as map_insert_scan, but the per-scan
 * work buffers (ray records, wave items, per-block counters; at most
 * 64 MiB) come from a fixed device array of the library, one per GPU, held
 * until the process ends, instead of buffers the map grows, and the call
 * enqueues kernels only (no allocation, no memset, no event).  The array is
 * shared by every map on the GPU: calls that overlap on one GPU (maps on
 * different streams) race and give wrong results; calls on one stream are
 * ordered and safe.  MAP_E_CAPACITY (map unchanged) when the scan needs more
 * than the array holds: about 16 + 8 * ceil(max(nx, ny, nz) / seg_len) / 64
 * bytes per point, so 2.7 M points on a 512 x 512 x 64 window at the default
 * seg_len of 8.
 * MAP_STATS_DISTINCT is not accepted (MAP_E_INVALID): its bitmaps are
 * allocated on first use.  map_get_stats reports the call's counters until
 * the next insert into the same map. */
int32_t map_insert_scan_static(map_t* m, const float* xyz_dev, int64_t n,
                               const float pose[12], uint32_t flags);

/* Writes the 2D maps of Sec. III-D into the caller's device arrays. *//* Writes the 2D maps of Sec. III-D into the caller's device arrays. */
int32_t map_export_2d(map_t* m, const map_2d_t* out_dev);

/* Writes the Sec. III-A lookup table and data array:
 *  lut_dev:   device int32[nx*ny*nz] (local linear index): rank of the voxel
 *             among occupied voxels (hits >= 1) in increasing index, else
 *             -1 - passes.
 *  data_dev:  device map_voxel_t[cap] in rank order; ranks >= cap are not
 *             written (cap may be 0 with data_dev NULL).
 *  n_occupied: host int64 receiving the number of occupied voxels M; written
 *             also when the data array is too small.
 *  origin_vox: host int32[3], receives the window origin (world voxel).
 * Synchronises the map's stream (to read M).  Returns MAP_E_CAPACITY when
 * cap < M: the table and the first cap entries are written and *n_occupied
 * holds M. */
int32_t map_export_voxels(map_t* m, int32_t* lut_dev, map_voxel_t* data_dev, int64_t cap,
                          int64_t* n_occupied, int32_t origin_vox[3]);

/* The same export without waiting: M goes to the DEVICE int64
 * n_occupied_dev (valid once the stream has been synchronised) and a data
 * array that is too small is not reported (the caller compares M with cap).
 * For pipelines that keep the host off the critical path. */
int32_t map_export_voxels_async(map_t* m, int32_t* lut_dev, map_voxel_t* data_dev, int64_t cap,
                                int64_t* n_occupied_dev, int32_t origin_vox[3]);

/* The voxel map itself as an output (Sec. I and Fig. 1, where denser voxels
 * are drawn more opaque; Sec. V): density_dev is a device float[nx*ny*nz] in
 * window-local linear order receiving, per voxel, hits / (hits + passes) for
 * an occupied voxel (the density of Sec. III-D, computed in double and
 * rounded once), 0 for a voxel rays only passed through, and the canonical
 * quiet NaN 0x7FC00000 for a voxel no ray reached.  Does not synchronise. */
int32_t map_export_density(map_t* m, float* density_dev);

/* Planner costmap (Sec. IV): each output map gets a weight and a pixel's cost
 * is the weighted sum of its layers.  Terms, added in this order in binary32:
 * slope, rough, density (each only where defined, i.e. not NaN), then the
 * weight of every flag layer the pixel has: positive obstacle, hard, soft,
 * negative obstacle, and `unknown` where the height is undefined.  Weights
 * must be finite (MAP_E_INVALID otherwise). */
typedef struct {
  float slope, rough, density, positive, hard, soft, negative, unknown;
} map_cost_weights_t;

/* in_dev: the 2D maps of m's window (as written by map_export_2d), cost_dev:
 * device float[nx][ny].  Enqueued on m's stream; reads no voxel state. */
int32_t map_costmap(map_t* m, const map_2d_t* in_dev, const map_cost_weights_t* w,
                    float* cost_dev);

/* Sets the map state from a lookup table and data array in the format above
 * (checkpoint / resume).  Every lut entry >= 0 must index data with hits >= 1,
 * and no entry may be INT32_MIN.  Synchronises; on invalid content the map
 * is left empty and MAP_E_INVALID is returned. */
int32_t map_import_voxels(map_t* m, const int32_t* lut_dev, const map_voxel_t* data_dev,
                          int64_t n_data, const int32_t origin_vox[3]);

/* Counters of the last insert; synchronises the map's stream. */
int32_t map_get_stats(map_t* m, map_stats_t* out);

/* Current window origin (world voxel index of window voxel (0,0,0)). */
int32_t map_get_origin(const map_t* m, int32_t origin_vox[3]);

/* Waits for the map's stream and returns the map's (sticky) status. */
int32_t map_sync(map_t* m);

/* Launch tuning (performance only: results are bit-identical for every
 * setting).  The traversal cuts every ray every seg_len dominant-axis voxels;
 * a wave takes one segment index of 64 rays of one ray-pass block (the block
 * groups its rays by segment count), counts its passes in an LDS table of
 * 64-byte map lines and adds each line to the map with one request; the
 * passes of a 17 x 17 x 9 box around the sensor are summed per block on chip
 * first.  seg_len: dominant-axis voxels per ray segment, 1..1024 (default 8);
 * trace_waves_per_cu: resident waves per compute unit requested for the
 * traversal grid (blocks of four waves), 1..32 (default 28, the most that fit
 * a compute unit); surface_tile: edge in
 * pixels of the tiles of the slope / roughness / negative-obstacle pass, 16
 * or 32 (default 32; other positive values are MAP_E_INVALID).  A field
 * <= 0 keeps the current value.  The batch autotuner sets all three. */
typedef struct {
  int32_t seg_len;
  int32_t trace_waves_per_cu;
  int32_t surface_tile;
} map_tuning_t;
int32_t map_set_tuning(map_t* m, const map_tuning_t* t);
int32_t map_get_tuning(const map_t* m, map_tuning_t* out);

/* Optional per-phase timing with HIP events recorded on the map's stream
 * around each kernel group (instrumentation for benchmarks).  Phases:
 * MAP_PROF_SCROLL (window clears), MAP_PROF_RAYS (transform, returns, ray
 * records and wave items), MAP_PROF_TRACE (ray traversal and sensor-box
 * fold), MAP_PROF_COLUMN (column
 * reduction), MAP_PROF_SURFACE (slope, roughness, negative obstacles),
 * MAP_PROF_LUT (lookup-table export).  map_profile_enable takes a mask (bit p
 * = phase p, 0 = off, MAP_PROF_ALL = every phase; each profiled phase costs
 * two event records per call).  map_profile_read synchronises, adds the
 * elapsed milliseconds and launch counts since the last read into
 * ms[MAP_PROF_N] / count[MAP_PROF_N] (host), and releases the events. */
#define MAP_PROF_SCROLL  0
#define MAP_PROF_RAYS    1
#define MAP_PROF_TRACE   2
#define MAP_PROF_COLUMN  3
#define MAP_PROF_SURFACE 4
#define MAP_PROF_LUT     5
#define MAP_PROF_N       6
#define MAP_PROF_ALL     ((1 << MAP_PROF_N) - 1)
int32_t map_profile_enable(map_t* m, int32_t phase_mask);
int32_t map_profile_read(map_t* m, double ms[MAP_PROF_N], int64_t count[MAP_PROF_N]);

/* ---- map buffer (Sec. III-B, III-C, III-D) --------------------------------
 * The paper's own dataflow.  Pointcloud processing turns each scan into a
 * voxel map of its own (a fresh window holding only that scan's hits, misses
 * and lowest returns, stored as a Sec. III-A lookup table + data array +
 * origin) and adds it to a buffer; map processing combines the buffered maps
 * into one map and computes the 2D maps from it.  The two sides run
 * asynchronously: pushes on the buffer's stream, the combine and the exports
 * on the output map's stream, ordered by events (a combine waits for the
 * pushes enqueued before it; a push waits for the combines enqueued before it,
 * which read the slot it overwrites).  Several lidars feed one buffer by
 * pushing their scans in turn. */
typedef struct map_buffer_t map_buffer_t;

/* Buffer of the `depth` (1..64) most recent per-scan maps of the window size
 * and resolution in `p`, in depth + 1 slots (the map the last push evicted is
 * kept until the next push), each holding a lookup table of the map's storage
 * size (4 bytes per voxel) and a data array of 12 bytes per occupied voxel
 * (grown to the largest scan pushed into it: a grow synchronises `stream`).
 * Pushes are enqueued on `stream` (NULL: the default stream). */
int32_t map_buffer_create(const map_params_t* p, int32_t depth, void* stream,
                          map_buffer_t** out);
/* Synchronises the buffer's stream and the combines still reading it. */
int32_t map_buffer_destroy(map_buffer_t* b);
/* Drops every buffered map and clears a sticky error (synchronises). */
int32_t map_buffer_reset(map_buffer_t* b);

/* Pointcloud processing of one scan (Sec. III-C) into the next slot,
 * replacing the oldest map once `depth` are held.  Arguments as in
 * map_insert_scan.  With MAP_RECENTER the scan's window is centred on its
 * pose; without it the scan takes the window of the newest buffered map (the
 * initial window while the buffer is empty), which is how a second lidar of
 * the same vehicle joins the primary lidar's map.  Errors as map_insert_scan
 * (the buffer is unchanged); MAP_E_OOM when a slot cannot grow. */
int32_t map_buffer_push(map_buffer_t* b, const float* xyz_dev, int64_t n, const float pose[12],
                        uint32_t flags);

/* Map processing, first step (Sec. III-D): replaces the state of `out` with
 * the combination of the buffered maps and sets its origin to the newest
 * buffered map's.  Every voxel of the new window is located in each buffered
 * map by the difference of the origins; where that map's window holds it,
 * its hits and misses are added and its lowest return (occupied voxels) takes
 * part in the minimum; voxels no buffered window holds are empty.  `out` must
 * have the buffer's nx, ny, nz and res_m (its other parameters govern its own
 * exports); map_export_2d / map_export_voxels then export the combined map.
 * Enqueued on out's stream.  MAP_E_INVALID when the buffer is empty. */
int32_t map_buffer_combine(map_buffer_t* b, map_t* out);

/* Combine strategy (results are identical): with `enable` (the default) a
 * combine into the same map as the previous combine of this buffer, made
 * exactly one push later and with that map unchanged in between, updates it
 * (adds the newest map, takes away the evicted one, recombines only the
 * voxels whose minimum could change and those that entered the window)
 * instead of combining every buffered map again; 0 always combines in full,
 * as the paper describes. */
int32_t map_buffer_set_incremental(map_buffer_t* b, int32_t enable);

/* Buffered maps (0..depth), or MAP_E_INVALID for a NULL buffer. */
int32_t map_buffer_count(const map_buffer_t* b);
/* Counters of the last push (as map_get_stats); synchronises the buffer's stream. */
int32_t map_buffer_get_stats(map_buffer_t* b, map_stats_t* out);

/* ---- batched serving (project extension, not in the paper) ---------------
 * Many vehicles' maps are stepped together: every stage of every map runs in
 * one persistent kernel per stage (grids sized to the device, walking the
 * maps' work from a descriptor table uploaded once per step), and the whole
 * step is captured once in a HIP graph and replayed. */
typedef struct map_batch_t map_batch_t;

/* Groups k distinct maps (1..64, created on the current device) for batched
 * steps enqueued on `stream` (NULL: the batch creates a stream of its own,
 * since graphs cannot be captured on the null stream).  A map may still be used by the single-map calls
 * between batch steps, never concurrently with one. */
int32_t map_batch_create(map_t* const* maps, int32_t k, void* stream, map_batch_t** out);
int32_t map_batch_destroy(map_batch_t* b);

/* One step: for every map i, the same results as map_insert_scan(maps[i],
 * xyz_dev[i], n[i], poses + 12*i, flags[i]) followed by map_export_2d(maps[i],
 * out2d + i) and, when lut_dev != NULL and lut_dev[i] != NULL,
 * map_export_voxels(maps[i], lut_dev[i], data_dev[i], cap[i],
 * n_occupied_dev[i], ...).  xyz_dev, n, poses, flags, out2d are arrays of k
 * (host arrays of device pointers where pointers); MAP_STATS_DISTINCT is not
 * accepted here.  Every request is checked before any map changes.
 * Synchronises (the per-map latencies are then available). */
int32_t map_batch_step(map_batch_t* b, const float* const* xyz_dev, const int64_t* n,
                       const float* poses, const uint32_t* flags, const map_2d_t* out2d,
                       int32_t* const* lut_dev, map_voxel_t* const* data_dev,
                       const int64_t* cap, int64_t* const* n_occupied_dev);

/* Latency of map i in the last step, ms: the device wall-clock time from the
 * start of the step to the end of map i's last kernel block.  ms[k]. */
int32_t map_batch_latency(const map_batch_t* b, double* ms);

/* Graph replay on (default) or off (plain stream launches of the same kernels). */
int32_t map_batch_set_graph(map_batch_t* b, int32_t enable);

/* Autotuner: times every candidate tuning (seg_len 6/8/16 x
 * trace_waves_per_cu 16/28 x surface_tile 16/32) on this step's inputs with
 * batch steps, applies
 * the fastest to all maps and appends it to the text cache `cache_path`
 * (NULL: no cache).  A cached entry for the same device, map shapes and
 * point-count range is applied without timing.  The maps are left empty
 * (map_reset) because the timing steps insert the inputs. */
int32_t map_batch_autotune(map_batch_t* b, const float* const* xyz_dev, const int64_t* n,
                           const float* poses, const uint32_t* flags, const map_2d_t* out2d,
                           const char* cache_path, map_tuning_t* chosen);

/* ---- learned gap-fill surrogate (project extension, not in the paper) -----
 * A 5-layer 3x3 convolution network (16 -> 32 -> 32 -> 32 -> 32 -> 2
 * channels, ReLU, zero padding; bf16 weights and layer inputs, fp32
 * accumulation, biases fp32) maps 16 per-column features to ground height and
 * roughness.  It never produces counts or flags: its output only fills
 * columns the plain method leaves undefined, through sgt_fill.  Images are
 * [H][W][C] device arrays with H = nx, W = ny of the map, channel fastest.
 * Parameters (fp32 master copy): per layer W[co][ci][ky][kx] then b[co]. */
typedef struct sgt_net_t sgt_net_t;

int64_t sgt_num_params(void);  /* 32962 */
/* Network for H x W images; He-normal weights from `seed`, zero biases,
 * identity normalisation.  Synchronises. */
int32_t sgt_create(int32_t H, int32_t W, uint64_t seed, void* stream, sgt_net_t** out);
int32_t sgt_destroy(sgt_net_t* n);
int32_t sgt_get_params(sgt_net_t* n, float* params_host);        /* synchronises */
int32_t sgt_set_params(sgt_net_t* n, const float* params_host);  /* synchronises */
/* Feature normalisation (x - mean) / std, computed in double and rounded to
 * float then bf16; mean[16], std[16] host, std > 0. */
int32_t sgt_set_norm(sgt_net_t* n, const float* mean, const float* std_dev);

/* Per-column features of map m (window-local [nx][ny][16], device): 0 sum of
 * hits, 1 sum of passes, 2 occupied voxels, 3 occupied fraction, 4 ground
 * height, 5 lowest return of the highest occupied voxel, 6 mean of the
 * occupied voxels' lowest returns, 7 height defined, 8 hits / (hits + passes)
 * of the ground voxel, 9 band density, 10 slope, 11 roughness, 12 slope
 * defined, 13 horizontal distance from the column centre to sensor_xyz, 14
 * sensor height above the ground, 15 column thinned (thin_dev[c] != 0; may be
 * NULL).  Undefined values are 0; a thinned column keeps only 13 and 15.
 * plain_dev: the map's map_export_2d output.  Heights in metres. */
int32_t sgt_features(map_t* m, const map_2d_t* plain_dev, const float sensor_xyz[3],
                     const uint8_t* thin_dev, float* feat_dev);
/* Removes the data of the window-local columns marked in thin_dev[nx*ny]. */
int32_t sgt_thin(map_t* m, const uint8_t* thin_dev);
/* sums[0..15] = per-feature sums, sums[16..31] = sums of squares (host). */
int32_t sgt_feature_sums(sgt_net_t* n, const float* feat_dev, double* sums_host);

/* out_dev[H][W][2] = network(features). */
int32_t sgt_forward(sgt_net_t* n, const float* feat_dev, float* out_dev);
/* Masked L1 loss against label_dev[H][W][2] (NaN = no label) and the gradient
 * of every parameter (kept for sgt_adam; also copied to grad_host if not
 * NULL).  The bf16 roundings are treated as the identity in the gradient.
 * Synchronises. */
int32_t sgt_loss_grad(sgt_net_t* n, const float* feat_dev, const float* label_dev,
                      float* loss_host, float* grad_host);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with the last gradient. */
int32_t sgt_adam(sgt_net_t* n, float lr);
/* Filled maps: the plain height / roughness where the plain height is
 * defined; elsewhere the network's (roughness clamped at 0) when the mean of
 * |network height - plain height| over the plain-defined columns of the
 * 11 x 11 window is <= tol_m; otherwise NaN. */
int32_t sgt_fill(const float* pred_dev, const map_2d_t* plain_dev, int32_t H, int32_t W,
                 float tol_m, float* height_out, float* rough_out, void* stream);

/* ---- roofline calibration (project measurement kernels) ------------------
 * The two reference rates the mapping kernels are priced against, measured on
 * the device at hand.  Both enqueue one kernel on `stream` and return without
 * waiting; the caller times them (HIP events) and owns every buffer.  They
 * are not part of the method. */

/* Plain device copy of `bytes` (a multiple of 16; both pointers 16-byte
 * aligned, the ranges disjoint) from src_dev to dst_dev: the practical HBM
 * rate, and the scale for hardware traffic counters (what they read for a
 * copy of known size).  MAP_E_INVALID on a null pointer or bad size or
 * alignment. */
int32_t map_calib_copy(void* dst_dev, const void* src_dev, int64_t bytes, void* stream);

/* Device-scope int32 atomic adds without return into target_dev[n_words]
 * (n_words a multiple of 16, at most 16 * (2^32 - 1)): n_waves waves (a
 * multiple of 4, at most 2^24) of 64 lanes each issue per_wave (1..4096)
 * instructions.  In every instruction each group of `lanes_per_line` lanes
 * (1, 2, 4, 8, 16 or 64) adds 1 to words of one pseudo-random 64-byte line
 * (a hash of seed, wave, instruction and group): distinct words for g <= 16,
 * four lanes on each of the 16 words for g = 64.  Updates in total:
 * 64 * n_waves * per_wave; line requests: that / lanes_per_line.  The sum of
 * target_dev grows by exactly the number of updates.  MAP_E_INVALID on a bad
 * argument. */
int32_t map_calib_atomic(int32_t* target_dev, int64_t n_words, int64_t n_waves,
                         int32_t per_wave, int32_t lanes_per_line, uint32_t seed, void* stream);

/* Static text for a status code. */
const char* map_status_str(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* GVOM_H */
