/*
 * gvom_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Interface of the plain, slow, single-threaded CPU oracle of the G-VOM
 * per-scan voxel-mapping path (Overbye & Saripalli, "G-VOM: A GPU Accelerated
 * Voxel Off-Road Mapping System", arXiv 2109.13176).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library: every type
 * below is declared here on its own.
 *
 * All pointers are host pointers.  Status codes: 0 ok, <0 error
 * (same numeric meaning as the product library's codes, defined here again).
 */
#ifndef GVOM_ORACLE_H
#define GVOM_ORACLE_H
#include <stdint.h>

#define ORC_OK              0
#define ORC_E_INVALID      -1
#define ORC_E_POSE         -2
#define ORC_E_SENSOR_OUT   -3
#define ORC_E_RANGE        -4
#define ORC_E_CAPACITY     -5
#define ORC_E_OOM          -6

#define ORC_RECENTER 1u

typedef struct {
  int32_t nx, ny, nz;
  float   res_m;
  int32_t sensor_z_voxel;
  float   obs_min_m, obs_max_m;
  int32_t dens_num, dens_den;
  int32_t fit_n;
  float   neg_thresh_m;
  float   neg_search_m;
} orc_params;

typedef struct {
  float   inv_r;
  int32_t n_lo, n_hi;
  int64_t tau_neg_q;
  int32_t search_d;
  int32_t half_fit;
} orc_consts;

typedef struct {
  int64_t n_points, n_nonfinite, n_range, n_hits, n_pass;
  int64_t n_distinct_pass, n_distinct_hit, n_cleared;
} orc_stats;

typedef struct orc_map orc_map;

int32_t orc_derive(const orc_params* p, orc_consts* c);
int32_t orc_create(const orc_params* p, orc_map** out);
void    orc_destroy(orc_map* m);
int32_t orc_reset(orc_map* m);
int32_t orc_insert_scan(orc_map* m, const float* xyz, int64_t n,
                        const float pose[12], uint32_t flags);
int32_t orc_export_2d(orc_map* m, float* height, float* slope, float* rough,
                      float* density, uint8_t* flags);
int32_t orc_export_voxels(orc_map* m, int32_t* lut, int32_t* data /* [cap][3] */,
                          int64_t cap, int64_t* n_occupied, int32_t origin[3]);
int32_t orc_import_voxels(orc_map* m, const int32_t* lut, const int32_t* data /* [n][3] */,
                          int64_t n_data, const int32_t origin[3]);
int32_t orc_combine(orc_map* out, int32_t k, const int32_t* const* luts,
                    const int32_t* const* datas /* [k] of [n][3] */,
                    const int32_t* origins /* [k][3], oldest first */);
int32_t orc_export_density(orc_map* m, float* density /* [nx*ny*nz] */);
int32_t orc_costmap(const float* slope, const float* rough, const float* density,
                    const uint8_t* flags, int64_t n, const double w[8], double* cost,
                    double* mag);
int32_t orc_get_stats(const orc_map* m, orc_stats* out);
int32_t orc_get_origin(const orc_map* m, int32_t origin[3]);

/* Building blocks exposed for the pins. */
int32_t orc_transform_point(const float pose[12], float inv_r, const float p[3],
                            int32_t q_out[3]);
int64_t orc_ray_voxels(const int32_t s_q[3], const int32_t p_q[3],
                       int32_t* out_xyz, int64_t cap);
int32_t orc_surface(const int32_t* hq, const uint8_t* defined, int32_t nx, int32_t ny,
                    int32_t fit_n, float res_m, int32_t search_d, int64_t tau_neg_q,
                    float* slope, float* rough, uint8_t* slope_def, uint8_t* negative);

#endif
