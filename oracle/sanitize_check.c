/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A standalone program that drives every entry point of the CPU oracle on
 * small seeded inputs, built with -fsanitize=address,undefined by the test
 * suite: a memory error or undefined behaviour anywhere in the oracle aborts
 * it.  It also checks invariants that hold for any input (returns equal the
 * in-window endpoints, ranks 0..M-1 in index order, a free voxel stores
 * -1 - passes, an export re-imported equals itself, flag exclusivity), so a
 * silent corruption fails too.  Prints "ok" and exits 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gvom_oracle.h"

int64_t orc_sgt_num_params(void);
int32_t orc_sgt_forward(const float* feat, int32_t H, int32_t W, const float* params,
                        int32_t round, double* out);
int32_t orc_sgt_loss_grad(const float* feat, int32_t H, int32_t W, const float* params,
                          const float* label, int32_t round, double* loss, double* grad);
int32_t orc_sgt_fill(const float* pred, const float* plain_h, const float* plain_r, int32_t H,
                     int32_t W, float tol_m, float* out_h, float* out_r);

#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
      exit(1);                                                          \
    }                                                                   \
  } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) {  /* xorshift64*, uniform in [0, 1) */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

static void cloud(float* xyz, int64_t n, float radius) {
  for (int64_t i = 0; i < n; i++) {
    for (int k = 0; k < 3; k++) xyz[3 * i + k] = (float)((2 * urand() - 1) * radius);
    const double u = urand();
    if (u < 0.03) xyz[3 * i + (i % 3)] = NAN;
    else if (u < 0.04) xyz[3 * i] = 1e30f;  /* out of range */
  }
}

static void pose_at(float pose[12], double yaw, double x, double y, double z) {
  const float c = (float)cos(yaw), s = (float)sin(yaw);
  const float P[12] = {c, -s, 0, (float)x, s, c, 0, (float)y, 0, 0, 1, (float)z};
  memcpy(pose, P, sizeof P);
}

typedef struct {
  int32_t* lut;
  int32_t* data;
  int64_t n;
  int32_t origin[3];
} export_t;

static export_t export_all(orc_map* m, int64_t V) {
  export_t e;
  e.lut = malloc((size_t)V * 4);
  e.data = malloc((size_t)V * 12);
  CHECK(e.lut && e.data);
  CHECK(orc_export_voxels(m, e.lut, e.data, V, &e.n, e.origin) == ORC_OK);
  return e;
}

static void check_export(const export_t* e, int64_t V) {
  int64_t rank = 0;
  for (int64_t i = 0; i < V; i++) {
    if (e->lut[i] >= 0) {
      CHECK(e->lut[i] == rank);
      CHECK(e->data[3 * rank] >= 1);
      rank++;
    } else {
      CHECK(-1 - e->lut[i] >= 0);
    }
  }
  CHECK(rank == e->n);
}

static void map_checks(const orc_params* p) {
  const int64_t V = (int64_t)p->nx * p->ny * p->nz, C = (int64_t)p->nx * p->ny;
  orc_map* m = NULL;
  CHECK(orc_create(p, &m) == ORC_OK);
  const int64_t n = 3000;
  float* xyz = malloc((size_t)n * 12);
  CHECK(xyz);
  float pose[12];
  int64_t hits_total = 0;
  for (int s = 0; s < 5; s++) {
    cloud(xyz, n, 0.6f * p->nx * p->res_m);
    pose_at(pose, 0.3 * s, 0.7 * s * p->res_m, -0.4 * s * p->res_m, 0.2 * s * p->res_m);
    CHECK(orc_insert_scan(m, xyz, n, pose, s % 2 ? ORC_RECENTER : 0) == ORC_OK);
    orc_stats st;
    CHECK(orc_get_stats(m, &st) == ORC_OK);
    CHECK(st.n_points == n && st.n_hits + st.n_nonfinite + st.n_range <= n);
    hits_total += st.n_hits;
  }
  /* error paths leave the map alone */
  pose[3] = NAN;
  CHECK(orc_insert_scan(m, xyz, n, pose, 0) == ORC_E_POSE);
  CHECK(orc_insert_scan(m, NULL, 5, pose, 0) == ORC_E_INVALID);
  pose_at(pose, 0.0, 1e7, 0, 0);
  CHECK(orc_insert_scan(m, xyz, n, pose, ORC_RECENTER) == ORC_E_RANGE);

  export_t e = export_all(m, V);
  check_export(&e, V);
  int64_t hsum = 0;
  for (int64_t r = 0; r < e.n; r++) hsum += e.data[3 * r];
  CHECK(hsum <= hits_total);
  /* a truncated export reports the capacity error and the full count */
  if (e.n > 1) {
    int32_t* lut2 = malloc((size_t)V * 4);
    int32_t* d2 = malloc((size_t)(e.n / 2) * 12 + 12);
    int64_t n2 = 0;
    int32_t o2[3];
    CHECK(lut2 && d2);
    CHECK(orc_export_voxels(m, lut2, d2, e.n / 2, &n2, o2) == ORC_E_CAPACITY);
    CHECK(n2 == e.n && memcmp(d2, e.data, (size_t)(e.n / 2) * 12) == 0);
    free(lut2);
    free(d2);
  }
  /* 2D export and its flag invariants */
  float *h = malloc((size_t)C * 4), *sl = malloc((size_t)C * 4), *ro = malloc((size_t)C * 4),
        *de = malloc((size_t)C * 4);
  uint8_t* fl = malloc((size_t)C);
  CHECK(h && sl && ro && de && fl);
  CHECK(orc_export_2d(m, h, sl, ro, de, fl) == ORC_OK);
  for (int64_t c = 0; c < C; c++) {
    const int def = (fl[c] & 1) != 0, pos = (fl[c] & 2) != 0, hard = (fl[c] & 4) != 0,
              soft = (fl[c] & 8) != 0, neg = (fl[c] & 16) != 0, sdef = (fl[c] & 32) != 0;
    CHECK(!(hard && soft));
    CHECK(!(hard || soft) || pos);
    CHECK(!neg || !def);
    CHECK(!pos || def);
    CHECK(!sdef || def);
    CHECK(def == !isnan(h[c]));
    CHECK(sdef == !isnan(sl[c]) && sdef == !isnan(ro[c]));
  }
  /* re-import: the same export comes back */
  orc_map* m2 = NULL;
  CHECK(orc_create(p, &m2) == ORC_OK);
  CHECK(orc_import_voxels(m2, e.lut, e.data, e.n, e.origin) == ORC_OK);
  export_t f = export_all(m2, V);
  CHECK(f.n == e.n && memcmp(f.lut, e.lut, (size_t)V * 4) == 0 &&
        memcmp(f.data, e.data, (size_t)e.n * 12) == 0);
  /* invalid content is rejected */
  if (e.n > 0) {
    int32_t* bad = malloc((size_t)V * 4);
    CHECK(bad);
    memcpy(bad, e.lut, (size_t)V * 4);
    bad[0] = (int32_t)e.n + 3;
    CHECK(orc_import_voxels(m2, bad, e.data, e.n, e.origin) == ORC_E_INVALID);
    free(bad);
  }
  /* density output, costmap, combine of two maps */
  float* dens = malloc((size_t)V * 4);
  CHECK(dens);
  CHECK(orc_export_density(m, dens) == ORC_OK);
  double w[8] = {1, 2, 3, 4, 5, 6, 7, 8};
  double* cost = malloc((size_t)C * 8);
  double* mag = malloc((size_t)C * 8);
  CHECK(cost && mag);
  CHECK(orc_costmap(sl, ro, de, fl, C, w, cost, mag) == ORC_OK);
  const int32_t* luts[2] = {e.lut, f.lut};
  const int32_t* datas[2] = {e.data, f.data};
  int32_t origins[6];
  memcpy(origins, e.origin, 12);
  memcpy(origins + 3, f.origin, 12);
  orc_map* out = NULL;
  CHECK(orc_create(p, &out) == ORC_OK);
  CHECK(orc_combine(out, 2, luts, datas, origins) == ORC_OK);
  export_t g = export_all(out, V);
  check_export(&g, V);
  CHECK(g.n == e.n);
  for (int64_t r = 0; r < g.n; r++) CHECK(g.data[3 * r] == 2 * e.data[3 * r]);
  CHECK(orc_reset(out) == ORC_OK);

  free(g.lut); free(g.data); free(f.lut); free(f.data); free(e.lut); free(e.data);
  free(h); free(sl); free(ro); free(de); free(fl); free(dens); free(cost); free(mag);
  free(xyz);
  orc_destroy(out);
  orc_destroy(m2);
  orc_destroy(m);
}

static void building_blocks(void) {
  orc_params p = {16, 16, 8, 0.5f, 4, 0.4f, 2.0f, 1, 2, 5, 0.5f, 5.0f};
  orc_consts c;
  CHECK(orc_derive(&p, &c) == ORC_OK);
  p.fit_n = 4;
  CHECK(orc_derive(&p, &c) == ORC_E_INVALID);
  float pose[12];
  pose_at(pose, 0.5, 1, 2, 3);
  const float pt[3] = {1.5f, -2.25f, 0.75f};
  int32_t q[3];
  CHECK(orc_transform_point(pose, 2.0f, pt, q) == 1);
  for (int r = 0; r < 200; r++) {
    int32_t s[3], e[3];
    for (int k = 0; k < 3; k++) {
      s[k] = (int32_t)((urand() * 2 - 1) * 20 * 65536);
      e[k] = (int32_t)((urand() * 2 - 1) * 20 * 65536);
      if (r % 4 == 0) e[k] &= ~0xFFFF;  /* lattice ties */
    }
    const int64_t len = orc_ray_voxels(s, e, NULL, 0);
    CHECK(len >= 1);
    int32_t* vox = malloc((size_t)len * 12);
    CHECK(vox);
    CHECK(orc_ray_voxels(s, e, vox, len) == len);
    for (int k = 0; k < 3; k++) {
      CHECK(vox[k] == (s[k] >> 16));
      CHECK(vox[3 * (len - 1) + k] == (e[k] >> 16));
    }
    free(vox);
  }
  const int nx = 24, ny = 20;
  int32_t* hq = malloc(nx * ny * 4);
  uint8_t* def = malloc(nx * ny);
  float *sl = malloc(nx * ny * 4), *ro = malloc(nx * ny * 4);
  uint8_t *sd = malloc(nx * ny), *ng = malloc(nx * ny);
  CHECK(hq && def && sl && ro && sd && ng);
  for (int i = 0; i < nx * ny; i++) {
    def[i] = urand() < 0.7;
    hq[i] = (int32_t)(urand() * 3 * 65536);
  }
  CHECK(orc_surface(hq, def, nx, ny, 5, 0.5f, 6, 65536, sl, ro, sd, ng) == ORC_OK);
  for (int i = 0; i < nx * ny; i++) CHECK(!(ng[i] && def[i]));
  free(hq); free(def); free(sl); free(ro); free(sd); free(ng);
}

static void surrogate(void) {
  const int H = 9, W = 7, F = 16;
  const int64_t P = orc_sgt_num_params();
  CHECK(P == 32962);
  float* feat = malloc((size_t)H * W * F * 4);
  float* prm = malloc((size_t)P * 4);
  float* label = malloc((size_t)H * W * 2 * 4);
  double* out = malloc((size_t)H * W * 2 * 8);
  double* grad = malloc((size_t)P * 8);
  CHECK(feat && prm && label && out && grad);
  for (int i = 0; i < H * W * F; i++) feat[i] = (float)(urand() * 2 - 1);
  for (int64_t i = 0; i < P; i++) prm[i] = (float)((urand() * 2 - 1) * 0.2);
  for (int i = 0; i < H * W * 2; i++) label[i] = urand() < 0.2 ? NAN : (float)urand();
  CHECK(orc_sgt_forward(feat, H, W, prm, 1, out) == 0);
  double loss = 0;
  CHECK(orc_sgt_loss_grad(feat, H, W, prm, label, 1, &loss, grad) == 0);
  CHECK(isfinite(loss) && loss >= 0);
  float *pred = malloc((size_t)H * W * 2 * 4), *ph = malloc(H * W * 4), *pr = malloc(H * W * 4);
  float *oh = malloc(H * W * 4), *orr = malloc(H * W * 4);
  CHECK(pred && ph && pr && oh && orr);
  for (int i = 0; i < H * W * 2; i++) pred[i] = (float)out[i];
  for (int i = 0; i < H * W; i++) {
    ph[i] = urand() < 0.5 ? NAN : (float)urand();
    pr[i] = (float)urand();
  }
  CHECK(orc_sgt_fill(pred, ph, pr, H, W, 0.05f, oh, orr) == 0);
  free(feat); free(prm); free(label); free(out); free(grad);
  free(pred); free(ph); free(pr); free(oh); free(orr);
}

int main(void) {
  const orc_params shapes[3] = {
      {24, 20, 12, 0.5f, 6, 0.4f, 2.0f, 1, 2, 5, 0.5f, 3.0f},
      {30, 34, 96, 0.1f, 48, 0.4f, 2.0f, 1, 2, 3, 0.5f, 1.0f},
      {16, 16, 16, 0.25f, 3, 0.2f, 1.0f, 2, 3, 7, 0.3f, 2.0f},
  };
  for (int i = 0; i < 3; i++) map_checks(&shapes[i]);
  building_blocks();
  surrogate();
  printf("ok\n");
  return 0;
}
