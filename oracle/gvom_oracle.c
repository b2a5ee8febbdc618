/*
 * gvom_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle).
 *
 * A plain, slow, single-threaded CPU statement of what the G-VOM per-scan
 * voxel-mapping path computes (arXiv 2109.13176, Section III).  It is written
 * for a reader who checks it against the paper, not for speed:
 *   - dense arrays in window coordinates, no toroidal addressing;
 *   - a ray's voxels come from sorting its exact boundary-crossing times;
 *   - the plane fit is the textbook normal-equation solve in double;
 *   - the negative-obstacle cones are enumerated cell by cell.
 * Only the tests, the smoke check and the CPU baseline of the benchmark load
 * this file.  It shares nothing with the HIP library.
 *
 * Fixed-point convention: a "Q" coordinate is a world coordinate in units of
 * 2^-16 voxel edge (int32).  Voxel index of a Q value = floor(Q / 65536).
 *
 * Parity unpinned: the whole-pipeline outputs on full synthetic scenes have no
 * independent reference; they are pinned piecewise (transform, ray voxels,
 * column rules, plane fit, cone search) by the tests under tests/.
 */
#include "gvom_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q_ONE 65536

struct orc_map {
  orc_params p;
  orc_consts c;
  int32_t origin[3];      /* world voxel index of window voxel (0,0,0) */
  int32_t *hits, *passes, *minqz;
  uint8_t *mark_pass, *mark_hit;
  orc_stats st;
};

/* ------------------------------------------------------------------------ */
/* Parameters and derived constants.  The paper names the map size and
 * resolution (III-A), the obstacle height band and density threshold (III-D),
 * the N x N fit window (III-D) and the negative-obstacle threshold and search
 * distance (III-D) but gives no values; they are inputs here.              */

int32_t orc_derive(const orc_params* p, orc_consts* c) {
  if (!p || !c) return ORC_E_INVALID;
  if (p->nx < 2 || p->ny < 2 || p->nz < 1) return ORC_E_INVALID;
  if ((p->nx % 2) || (p->ny % 2)) return ORC_E_INVALID;
  if (p->nx > 8192 || p->ny > 8192 || p->nz > 128) return ORC_E_INVALID;
  if ((double)p->nx * (double)p->ny * (double)p->nz > 2147483647.0) return ORC_E_INVALID;
  if (!(p->res_m > 0.0f) || !isfinite(p->res_m)) return ORC_E_INVALID;
  if (p->sensor_z_voxel < 0 || p->sensor_z_voxel >= p->nz) return ORC_E_INVALID;
  if (!isfinite(p->obs_min_m) || !isfinite(p->obs_max_m) || p->obs_min_m < 0.0f ||
      p->obs_max_m < p->obs_min_m) return ORC_E_INVALID;
  if (p->dens_den <= 0 || p->dens_num < 0) return ORC_E_INVALID;
  if (p->fit_n < 3 || p->fit_n > 15 || (p->fit_n % 2) == 0) return ORC_E_INVALID;
  if (!isfinite(p->neg_thresh_m) || p->neg_thresh_m < 0.0f) return ORC_E_INVALID;
  if (!isfinite(p->neg_search_m) || p->neg_search_m < 0.0f) return ORC_E_INVALID;

  double r = (double)p->res_m;
  c->inv_r = (float)(1.0 / r);
  long lo = lround((double)p->obs_min_m / r);  /* lround: half away from zero */
  c->n_lo = (int32_t)(lo < 1 ? 1 : lo);
  c->n_hi = (int32_t)lround((double)p->obs_max_m / r);
  c->tau_neg_q = (int64_t)floor((double)p->neg_thresh_m / r * 65536.0);
  c->search_d = (int32_t)lround((double)p->neg_search_m / r);
  c->half_fit = (p->fit_n - 1) / 2;
  if (c->n_hi < c->n_lo) return ORC_E_INVALID;
  if (c->search_d < 1 || c->search_d > 64) return ORC_E_INVALID;
  return ORC_OK;
}

static int64_t n_vox(const orc_map* m) {
  return (int64_t)m->p.nx * m->p.ny * m->p.nz;
}

/* Window-local voxel (x, y, z) -> linear index, z fastest (III-A: the lookup
 * table is a 3D array the size of the map). */
static int64_t lin(const orc_map* m, int64_t x, int64_t y, int64_t z) {
  return (x * m->p.ny + y) * m->p.nz + z;
}

static int inside(const orc_map* m, int64_t x, int64_t y, int64_t z) {
  return x >= 0 && x < m->p.nx && y >= 0 && y < m->p.ny && z >= 0 && z < m->p.nz;
}

static void make_empty(orc_map* m, int64_t i) {
  m->hits[i] = 0;
  m->passes[i] = 0;
  m->minqz[i] = INT32_MAX;
}

int32_t orc_create(const orc_params* p, orc_map** out) {
  if (!out) return ORC_E_INVALID;
  *out = NULL;
  orc_consts c;
  int32_t s = orc_derive(p, &c);
  if (s) return s;
  orc_map* m = (orc_map*)calloc(1, sizeof(orc_map));
  if (!m) return ORC_E_OOM;
  m->p = *p;
  m->c = c;
  int64_t v = n_vox(m);
  m->hits = (int32_t*)malloc(sizeof(int32_t) * v);
  m->passes = (int32_t*)malloc(sizeof(int32_t) * v);
  m->minqz = (int32_t*)malloc(sizeof(int32_t) * v);
  m->mark_pass = (uint8_t*)malloc(v);
  m->mark_hit = (uint8_t*)malloc(v);
  if (!m->hits || !m->passes || !m->minqz || !m->mark_pass || !m->mark_hit) {
    orc_destroy(m);
    return ORC_E_OOM;
  }
  orc_reset(m);
  *out = m;
  return ORC_OK;
}

void orc_destroy(orc_map* m) {
  if (!m) return;
  free(m->hits);
  free(m->passes);
  free(m->minqz);
  free(m->mark_pass);
  free(m->mark_hit);
  free(m);
}

/* Empty map.  Until the first recentring the window is placed so that the
 * world origin falls in voxel (nx/2, ny/2, sensor_z_voxel). */
int32_t orc_reset(orc_map* m) {
  if (!m) return ORC_E_INVALID;
  for (int64_t i = 0; i < n_vox(m); i++) make_empty(m, i);
  m->origin[0] = -m->p.nx / 2;
  m->origin[1] = -m->p.ny / 2;
  m->origin[2] = -m->p.sensor_z_voxel;
  memset(&m->st, 0, sizeof(m->st));
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-C: the odometry transforms the cloud into the map frame.  Pose is the
 * sensor-to-world [R | t], row-major 3x4.  Each coordinate is one chain of
 * fused multiply-adds in the order t, x, y, z; then scaled to voxel units and
 * quantised to Q16 by floor.  Returns 1 if the point is usable, 0 if it must
 * be skipped (non-finite input or result, or |u| >= 2^15 voxels).          */
int32_t orc_transform_point(const float pose[12], float inv_r, const float p[3],
                            int32_t q_out[3]) {
  for (int i = 0; i < 3; i++)
    if (!isfinite(p[i])) return 0;
  for (int i = 0; i < 3; i++) {
    float w = pose[4 * i + 3];
    w = fmaf(pose[4 * i + 0], p[0], w);
    w = fmaf(pose[4 * i + 1], p[1], w);
    w = fmaf(pose[4 * i + 2], p[2], w);
    if (!isfinite(w)) return 0;
    float u = w * inv_r;
    if (!(fabsf(u) < 32768.0f)) return 0;
    q_out[i] = (int32_t)floorf(u * 65536.0f);
  }
  return 1;
}

/* floor(q / 65536) written out in double, exact for every int32. */
static int32_t vox_of(int64_t q) { return (int32_t)floor((double)q / 65536.0); }

/* ------------------------------------------------------------------------ */
/* III-A / III-C: a ray "passes" every voxel it crosses without ending in it.
 * The ray is the segment X(t) = S + t (P - S), t in [0, 1], in Q units.  Its
 * voxels are the distinct values of floor(X(t) / 65536) in increasing t.
 *
 * Here this definition is evaluated directly: every boundary crossing of
 * every axis is an event at an exact rational time; the events are sorted;
 * at a common time, axes moving up enter their new cell AT that time (the
 * boundary belongs to the upper cell) and axes moving down leave their cell
 * just AFTER it, so the voxel at the time itself is emitted between the two.
 * Writes the voxel sequence (x, y, z triples) and returns its length.       */
typedef struct {
  int64_t num, den; /* time = num / den, den > 0 */
  int axis, dir;
} crossing;

static int cmp_crossing(const void* a, const void* b) {
  const crossing* u = (const crossing*)a;
  const crossing* v = (const crossing*)b;
  __int128 l = (__int128)u->num * v->den;
  __int128 r = (__int128)v->num * u->den;
  return (l < r) ? -1 : (l > r) ? 1 : 0;
}

static int same_time(const crossing* u, const crossing* v) {
  return (__int128)u->num * v->den == (__int128)v->num * u->den;
}

int64_t orc_ray_voxels(const int32_t s_q[3], const int32_t p_q[3], int32_t* out_xyz,
                       int64_t cap) {
  int64_t total = 0;
  for (int a = 0; a < 3; a++) {
    int64_t d = (int64_t)vox_of(p_q[a]) - vox_of(s_q[a]);
    total += d < 0 ? -d : d;
  }
  crossing* ev = (crossing*)malloc(sizeof(crossing) * (size_t)(total > 0 ? total : 1));
  if (!ev) return -1;
  int64_t ne = 0;
  for (int a = 0; a < 3; a++) {
    int64_t S = s_q[a], P = p_q[a], D = P - S;
    int64_t c0 = vox_of(S), c1 = vox_of(P);
    if (c1 > c0) {
      for (int64_t k = 1; k <= c1 - c0; k++) {
        int64_t b = (c0 + k) * Q_ONE; /* boundary entered when X reaches b */
        ev[ne].num = b - S;
        ev[ne].den = D;
        ev[ne].axis = a;
        ev[ne].dir = +1;
        ne++;
      }
    } else if (c1 < c0) {
      for (int64_t k = 1; k <= c0 - c1; k++) {
        int64_t b = (c0 - k + 1) * Q_ONE; /* lower face of the current cell */
        ev[ne].num = S - b;
        ev[ne].den = -D;
        ev[ne].axis = a;
        ev[ne].dir = -1;
        ne++;
      }
    }
  }
  qsort(ev, (size_t)ne, sizeof(crossing), cmp_crossing);

  int32_t v[3] = {vox_of(s_q[0]), vox_of(s_q[1]), vox_of(s_q[2])};
  int64_t n = 0;
#define EMIT()                                         \
  do {                                                 \
    if (n < cap) {                                     \
      out_xyz[3 * n + 0] = v[0];                       \
      out_xyz[3 * n + 1] = v[1];                       \
      out_xyz[3 * n + 2] = v[2];                       \
    }                                                  \
    n++;                                               \
  } while (0)
  EMIT();
  int64_t i = 0;
  while (i < ne) {
    int64_t j = i;
    while (j < ne && same_time(&ev[i], &ev[j])) j++;
    int up = 0, down = 0;
    for (int64_t k = i; k < j; k++)
      if (ev[k].dir > 0) {
        v[ev[k].axis] += 1;
        up = 1;
      }
    if (up) EMIT();
    for (int64_t k = i; k < j; k++)
      if (ev[k].dir < 0) {
        v[ev[k].axis] -= 1;
        down = 1;
      }
    if (down) EMIT();
    i = j;
  }
#undef EMIT
  free(ev);
  return n;
}

/* ------------------------------------------------------------------------ */
/* The window follows the vehicle.  Its origin is always a whole number of
 * voxels (III-A), so a voxel keeps its world cell when the window moves; a
 * voxel present in both the old and the new window keeps its data, every
 * other voxel of the new window starts empty.                             */
static int32_t move_window(orc_map* m, const int32_t new_origin[3]) {
  if (new_origin[0] == m->origin[0] && new_origin[1] == m->origin[1] &&
      new_origin[2] == m->origin[2])
    return ORC_OK;
  int64_t v = n_vox(m);
  int32_t* h = (int32_t*)malloc(sizeof(int32_t) * v);
  int32_t* ps = (int32_t*)malloc(sizeof(int32_t) * v);
  int32_t* mq = (int32_t*)malloc(sizeof(int32_t) * v);
  if (!h || !ps || !mq) {
    free(h);
    free(ps);
    free(mq);
    return ORC_E_OOM;
  }
  int64_t cleared = 0;
  for (int64_t x = 0; x < m->p.nx; x++)
    for (int64_t y = 0; y < m->p.ny; y++)
      for (int64_t z = 0; z < m->p.nz; z++) {
        int64_t i = lin(m, x, y, z);
        int64_t ox = x + new_origin[0] - m->origin[0];
        int64_t oy = y + new_origin[1] - m->origin[1];
        int64_t oz = z + new_origin[2] - m->origin[2];
        if (inside(m, ox, oy, oz)) {
          int64_t j = lin(m, ox, oy, oz);
          h[i] = m->hits[j];
          ps[i] = m->passes[j];
          mq[i] = m->minqz[j];
        } else {
          h[i] = 0;
          ps[i] = 0;
          mq[i] = INT32_MAX;
          cleared++;
        }
      }
  free(m->hits);
  free(m->passes);
  free(m->minqz);
  m->hits = h;
  m->passes = ps;
  m->minqz = mq;
  m->origin[0] = new_origin[0];
  m->origin[1] = new_origin[1];
  m->origin[2] = new_origin[2];
  m->st.n_cleared = cleared;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-C pointcloud processing for one scan: transform, then for each ray the
 * return is counted in its end voxel together with the lowest return height,
 * and every other voxel on the ray counts one pass (III-A metrics).  Rays are
 * independent and every update is an addition or a minimum, so the result
 * does not depend on point order.                                          */
int32_t orc_insert_scan(orc_map* m, const float* xyz, int64_t n, const float pose[12],
                        uint32_t flags) {
  if (!m || !pose || n < 0 || (n > 0 && !xyz)) return ORC_E_INVALID;
  if (flags & ~ORC_RECENTER) return ORC_E_INVALID;
  for (int i = 0; i < 12; i++)
    if (!isfinite(pose[i])) return ORC_E_POSE;
  int32_t S[3];
  for (int i = 0; i < 3; i++) {
    float u = pose[4 * i + 3] * m->c.inv_r;
    if (!(fabsf(u) < 32768.0f)) return ORC_E_RANGE;
    S[i] = (int32_t)floorf(u * 65536.0f);
  }
  int32_t sv[3] = {vox_of(S[0]), vox_of(S[1]), vox_of(S[2])};
  memset(&m->st, 0, sizeof(m->st));
  if (flags & ORC_RECENTER) {
    int32_t o[3] = {sv[0] - m->p.nx / 2, sv[1] - m->p.ny / 2, sv[2] - m->p.sensor_z_voxel};
    int32_t s = move_window(m, o);
    if (s) return s;
  } else if (!inside(m, (int64_t)sv[0] - m->origin[0], (int64_t)sv[1] - m->origin[1],
                     (int64_t)sv[2] - m->origin[2])) {
    return ORC_E_SENSOR_OUT;
  }
  int64_t v = n_vox(m);
  memset(m->mark_pass, 0, (size_t)v);
  memset(m->mark_hit, 0, (size_t)v);
  m->st.n_points = n;

  int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * 3 * 8192);
  if (!seq) return ORC_E_OOM;
  for (int64_t k = 0; k < n; k++) {
    int finite = isfinite(xyz[3 * k]) && isfinite(xyz[3 * k + 1]) && isfinite(xyz[3 * k + 2]);
    int32_t Q[3];
    if (!finite) {
      m->st.n_nonfinite++;
      continue;
    }
    if (!orc_transform_point(pose, m->c.inv_r, &xyz[3 * k], Q)) {
      m->st.n_range++;
      continue;
    }
    int far = 0;
    for (int a = 0; a < 3; a++) {
      int64_t d = (int64_t)Q[a] - S[a];
      if (d >= (1 << 27) || -d >= (1 << 27)) far = 1;
    }
    if (far) {
      m->st.n_range++;
      continue;
    }
    /* the return: hit count and lowest return height of the end voxel */
    int64_t ex = (int64_t)vox_of(Q[0]) - m->origin[0];
    int64_t ey = (int64_t)vox_of(Q[1]) - m->origin[1];
    int64_t ez = (int64_t)vox_of(Q[2]) - m->origin[2];
    if (inside(m, ex, ey, ez)) {
      int64_t i = lin(m, ex, ey, ez);
      m->hits[i] += 1;
      if (Q[2] < m->minqz[i]) m->minqz[i] = Q[2];
      m->st.n_hits++;
      if (!m->mark_hit[i]) {
        m->mark_hit[i] = 1;
        m->st.n_distinct_hit++;
      }
    }
    /* the passes: every voxel of the ray but the last, inside the window */
    int64_t len = orc_ray_voxels(S, Q, seq, 8192);
    if (len < 1 || len > 8192) {
      free(seq);
      return ORC_E_OOM;
    }
    for (int64_t j = 0; j + 1 < len; j++) {
      int64_t x = (int64_t)seq[3 * j] - m->origin[0];
      int64_t y = (int64_t)seq[3 * j + 1] - m->origin[1];
      int64_t z = (int64_t)seq[3 * j + 2] - m->origin[2];
      if (!inside(m, x, y, z)) continue;
      int64_t i = lin(m, x, y, z);
      m->passes[i] += 1;
      m->st.n_pass++;
      if (!m->mark_pass[i]) {
        m->mark_pass[i] = 1;
        m->st.n_distinct_pass++;
      }
    }
  }
  free(seq);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-D slope and roughness: least-squares plane z = a dx + b dy + c over the
 * defined heights of the N x N pixel square around a defined pixel (cut at
 * the map edge), heights relative to the centre; slope = |(a, b)| as rise
 * over run; roughness = mean squared residual in m^2.  The fit is defined
 * when at least 3 heights take part and the (integer) normal matrix is
 * non-singular.
 *
 * III-D negative obstacles: for a pixel without a height, four quadrant cones
 * (+x, -x, +y, -y; diagonals shared) each grow ring by ring up to D pixels
 * and stop at the first ring slice holding a defined in-map cell; all defined
 * cells of the stopping slices form one set; the pixel is negative when that
 * set has two or more cells and max - min of their heights exceeds the
 * threshold.                                                               */
/* Solves A x = b by Gaussian elimination with partial pivoting. */
static void solve3(double A[3][3], double b[3], double x[3]) {
  for (int col = 0; col < 3; col++) {
    int piv = col;
    for (int r = col + 1; r < 3; r++)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col) {
      for (int k = 0; k < 3; k++) {
        double t = A[col][k];
        A[col][k] = A[piv][k];
        A[piv][k] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < 3; r++) {
      double f = A[r][col] / A[col][col];
      for (int k = col; k < 3; k++) A[r][k] -= f * A[col][k];
      b[r] -= f * b[col];
    }
  }
  for (int r = 2; r >= 0; r--) {
    double s = b[r];
    for (int k = r + 1; k < 3; k++) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
}

static float qnan(void) {
  union {
    uint32_t u;
    float f;
  } v;
  v.u = 0x7FC00000u;
  return v.f;
}

int32_t orc_surface(const int32_t* hq, const uint8_t* defined, int32_t nx, int32_t ny,
                    int32_t fit_n, float res_m, int32_t search_d, int64_t tau_neg_q,
                    float* slope, float* rough, uint8_t* slope_def, uint8_t* negative) {
  if (!hq || !defined || !slope || !rough || !slope_def || !negative) return ORC_E_INVALID;
  if (nx < 1 || ny < 1 || fit_n < 3 || (fit_n % 2) == 0) return ORC_E_INVALID;
  int h = (fit_n - 1) / 2;
  double q2m = (double)res_m / 65536.0;
  for (int64_t i = 0; i < nx; i++)
    for (int64_t j = 0; j < ny; j++) {
      int64_t c = i * ny + j;
      slope[c] = qnan();
      rough[c] = qnan();
      slope_def[c] = 0;
      negative[c] = 0;
      if (defined[c]) {
        /* plane fit */
        int64_t n = 0, sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
        double A[3][3] = {{0}}, b[3] = {0};
        for (int64_t dx = -h; dx <= h; dx++)
          for (int64_t dy = -h; dy <= h; dy++) {
            int64_t x = i + dx, y = j + dy;
            if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
            if (!defined[x * ny + y]) continue;
            double dz = (double)((int64_t)hq[x * ny + y] - hq[c]);
            n++;
            sx += dx;
            sy += dy;
            sxx += dx * dx;
            syy += dy * dy;
            sxy += dx * dy;
            double row[3] = {(double)dx, (double)dy, 1.0};
            for (int r = 0; r < 3; r++) {
              for (int k = 0; k < 3; k++) A[r][k] += row[r] * row[k];
              b[r] += row[r] * dz;
            }
          }
        /* exact determinant of the integer normal matrix decides definedness */
        int64_t det = sxx * (syy * n - sy * sy) - sxy * (sxy * n - sy * sx) +
                      sx * (sxy * sy - syy * sx);
        if (n >= 3 && det != 0) {
          double x[3];
          solve3(A, b, x);
          double ss = 0.0;
          for (int64_t dx = -h; dx <= h; dx++)
            for (int64_t dy = -h; dy <= h; dy++) {
              int64_t xx = i + dx, yy = j + dy;
              if (xx < 0 || xx >= nx || yy < 0 || yy >= ny) continue;
              if (!defined[xx * ny + yy]) continue;
              double dz = (double)((int64_t)hq[xx * ny + yy] - hq[c]);
              double e = dz - (x[0] * dx + x[1] * dy + x[2]);
              ss += e * e;
            }
          slope[c] = (float)(sqrt(x[0] * x[0] + x[1] * x[1]) / 65536.0);
          rough[c] = (float)(ss / (double)n * q2m * q2m);
          slope_def[c] = 1;
        }
      } else {
        /* cone search */
        int64_t found = 0, lo = INT64_MAX, hi = INT64_MIN;
        for (int cone = 0; cone < 4; cone++) {
          for (int64_t d = 1; d <= search_d; d++) {
            int any = 0;
            for (int64_t e = -d; e <= d; e++) {
              int64_t x, y;
              if (cone == 0) { x = i + d; y = j + e; }
              else if (cone == 1) { x = i - d; y = j + e; }
              else if (cone == 2) { x = i + e; y = j + d; }
              else { x = i + e; y = j - d; }
              if (x < 0 || x >= nx || y < 0 || y >= ny) continue;
              if (!defined[x * ny + y]) continue;
              any = 1;
              int64_t v = hq[x * ny + y];
              found++;
              if (v < lo) lo = v;
              if (v > hi) hi = v;
            }
            if (any) break;
          }
        }
        /* a diagonal cell may be counted by two cones; that cannot change
           max - min, and max - min > tau >= 0 needs two distinct cells */
        if (found >= 2 && hi - lo > tau_neg_q) negative[c] = 1;
      }
    }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-D 2D maps from the voxel map.
 *  height: lowest return of the lowest occupied voxel of the column;
 *  positive obstacle: an occupied voxel from n_lo to n_hi voxels above the
 *    ground voxel; density of the band = sum(hits) / sum(hits + passes) over
 *    its occupied voxels; hard when density > num/den, else soft;
 *  slope, roughness, negative obstacles: orc_surface.
 * flags: bit0 height, bit1 positive, bit2 hard, bit3 soft, bit4 negative,
 * bit5 slope defined.  Undefined floats are the quiet NaN 0x7FC00000.      */
int32_t orc_export_2d(orc_map* m, float* height, float* slope, float* rough,
                      float* density, uint8_t* flags) {
  if (!m || !height || !slope || !rough || !density || !flags) return ORC_E_INVALID;
  int64_t nx = m->p.nx, ny = m->p.ny, nz = m->p.nz;
  int64_t C = nx * ny;
  int32_t* hq = (int32_t*)malloc(sizeof(int32_t) * C);
  uint8_t* def = (uint8_t*)malloc(C);
  uint8_t* sdef = (uint8_t*)malloc(C);
  uint8_t* neg = (uint8_t*)malloc(C);
  if (!hq || !def || !sdef || !neg) {
    free(hq);
    free(def);
    free(sdef);
    free(neg);
    return ORC_E_OOM;
  }
  double r = (double)m->p.res_m;
  for (int64_t x = 0; x < nx; x++)
    for (int64_t y = 0; y < ny; y++) {
      int64_t c = x * ny + y;
      uint8_t f = 0;
      int64_t kg = -1;
      for (int64_t z = 0; z < nz; z++)
        if (m->hits[lin(m, x, y, z)] >= 1) {
          kg = z;
          break;
        }
      height[c] = qnan();
      density[c] = qnan();
      hq[c] = 0;
      def[c] = 0;
      if (kg >= 0) {
        int32_t q = m->minqz[lin(m, x, y, kg)];
        hq[c] = q;
        def[c] = 1;
        height[c] = (float)((double)q * r / 65536.0);
        f |= 1;
        int64_t sh = 0, sa = 0, cnt = 0;
        for (int64_t z = kg + m->c.n_lo; z <= kg + m->c.n_hi && z < nz; z++) {
          int64_t i = lin(m, x, y, z);
          if (m->hits[i] >= 1) {
            sh += m->hits[i];
            sa += (int64_t)m->hits[i] + m->passes[i];
            cnt++;
          }
        }
        if (cnt > 0) {
          f |= 2;
          density[c] = (float)((double)sh / (double)sa);
          if (sh * m->p.dens_den > (int64_t)m->p.dens_num * sa)
            f |= 4;
          else
            f |= 8;
        }
      }
      flags[c] = f;
    }
  orc_surface(hq, def, m->p.nx, m->p.ny, m->p.fit_n, m->p.res_m, m->c.search_d,
              m->c.tau_neg_q, slope, rough, sdef, neg);
  for (int64_t c = 0; c < C; c++) {
    if (sdef[c]) flags[c] |= 32;
    if (neg[c]) flags[c] |= 16;
  }
  free(hq);
  free(def);
  free(sdef);
  free(neg);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-A storage: the lookup table holds, for an occupied voxel, its index in
 * the data array and otherwise -1 - (number of passes).  The data array is
 * ordered by increasing lookup-table index (one valid order; the paper allows
 * any).  Each entry: hits, passes, lowest return (Q).  Entries at rank >= cap
 * are not written; n_occupied is always written.                          */
int32_t orc_export_voxels(orc_map* m, int32_t* lut, int32_t* data, int64_t cap,
                          int64_t* n_occupied, int32_t origin[3]) {
  if (!m || !lut || !n_occupied || !origin || cap < 0 || (cap > 0 && !data))
    return ORC_E_INVALID;
  int64_t rank = 0;
  for (int64_t i = 0; i < n_vox(m); i++) {
    if (m->hits[i] >= 1) {
      lut[i] = (int32_t)rank;
      if (rank < cap) {
        data[3 * rank + 0] = m->hits[i];
        data[3 * rank + 1] = m->passes[i];
        data[3 * rank + 2] = m->minqz[i];
      }
      rank++;
    } else {
      lut[i] = -1 - m->passes[i];
    }
  }
  *n_occupied = rank;
  origin[0] = m->origin[0];
  origin[1] = m->origin[1];
  origin[2] = m->origin[2];
  return rank > cap ? ORC_E_CAPACITY : ORC_OK;
}

/* Inverse of the export: the window state is set from a lookup table and data
 * array in the III-A format (used to build hand-filled maps in the tests). */
int32_t orc_import_voxels(orc_map* m, const int32_t* lut, const int32_t* data,
                          int64_t n_data, const int32_t origin[3]) {
  if (!m || !lut || !origin || n_data < 0 || (n_data > 0 && !data)) return ORC_E_INVALID;
  for (int64_t i = 0; i < n_vox(m); i++) {
    if (lut[i] >= 0) {
      if (lut[i] >= n_data || data[3 * (int64_t)lut[i]] < 1) return ORC_E_INVALID;
    } else if (lut[i] == INT32_MIN) {
      return ORC_E_INVALID;
    }
  }
  for (int64_t i = 0; i < n_vox(m); i++) {
    if (lut[i] >= 0) {
      const int32_t* d = &data[3 * (int64_t)lut[i]];
      m->hits[i] = d[0];
      m->passes[i] = d[1];
      m->minqz[i] = d[2];
    } else {
      m->hits[i] = 0;
      m->passes[i] = -1 - lut[i];
      m->minqz[i] = INT32_MAX;
    }
  }
  m->origin[0] = origin[0];
  m->origin[1] = origin[1];
  m->origin[2] = origin[2];
  memset(&m->st, 0, sizeof(m->st));
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* III-B / III-D: map processing starts by combining the buffered per-scan
 * maps (each a III-A lookup table + data array + origin, in the format that
 * orc_export_voxels writes) into one map.  The combined map takes the origin
 * of the most recent buffered map, which is the last one given.  Every voxel
 * of the combined window is looked up in each buffered map by offsetting its
 * index with the difference of the two origins; where that map's window holds
 * the voxel, hits and misses are added (the misses of a free voxel are
 * -1 - lut) and, for an occupied entry, its lowest return takes part in the
 * minimum.  Voxels that no buffered window holds are empty.  The window size
 * of every buffered map is the one of `out`.                                */
int32_t orc_combine(orc_map* out, int32_t k, const int32_t* const* luts,
                    const int32_t* const* datas, const int32_t* origins) {
  if (!out || k < 1 || !luts || !datas || !origins) return ORC_E_INVALID;
  const int32_t* o = &origins[3 * (k - 1)];
  for (int64_t x = 0; x < out->p.nx; x++)
    for (int64_t y = 0; y < out->p.ny; y++)
      for (int64_t z = 0; z < out->p.nz; z++) {
        int32_t hits = 0, passes = 0, minqz = INT32_MAX;
        for (int32_t j = 0; j < k; j++) {
          const int32_t* oj = &origins[3 * j];
          /* the same world voxel, in window coordinates of buffered map j */
          const int64_t xj = o[0] + x - oj[0], yj = o[1] + y - oj[1], zj = o[2] + z - oj[2];
          if (!inside(out, xj, yj, zj)) continue;
          const int32_t e = luts[j][lin(out, xj, yj, zj)];
          if (e >= 0) {
            const int32_t* d = &datas[j][3 * (int64_t)e];
            hits += d[0];
            passes += d[1];
            if (d[2] < minqz) minqz = d[2];
          } else {
            passes += -1 - e;
          }
        }
        const int64_t i = lin(out, x, y, z);
        out->hits[i] = hits;
        out->passes[i] = passes;
        out->minqz[i] = minqz;
      }
  out->origin[0] = o[0];
  out->origin[1] = o[1];
  out->origin[2] = o[2];
  memset(&out->st, 0, sizeof(out->st));
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The completed voxel map is an output of its own (Sec. I, Fig. 1, where it
 * is drawn more opaque where denser; Sec. V).  Per voxel of the window, in
 * lookup-table order: an occupied voxel has the density hits / (hits +
 * passes) that III-D uses for obstacle bands; a voxel that rays only passed
 * through has 0; a voxel no ray reached is unobserved (NaN).               */
int32_t orc_export_density(orc_map* m, float* density) {
  if (!m || !density) return ORC_E_INVALID;
  for (int64_t i = 0; i < n_vox(m); i++) {
    if (m->hits[i] >= 1)
      density[i] = (float)((double)m->hits[i] / ((double)m->hits[i] + (double)m->passes[i]));
    else if (m->passes[i] >= 1)
      density[i] = 0.0f;
    else
      density[i] = qnan();
  }
  return ORC_OK;
}

/* Sec. IV: the planner's costmap gives each output map a weight; a pixel's
 * cost is the weighted sum of its layers.  Layers, in the order of w[]:
 * slope, roughness, density (each where defined, else no term), then the
 * indicator layers positive obstacle, hard, soft, negative obstacle and
 * unknown ground (height undefined), from the flag bits of the 2D export.
 * cost[i] is the sum in double; mag[i] = sum of the terms' magnitudes. */
int32_t orc_costmap(const float* slope, const float* rough, const float* density,
                    const uint8_t* flags, int64_t n, const double w[8], double* cost,
                    double* mag) {
  if (!slope || !rough || !density || !flags || n < 0 || !w || !cost || !mag)
    return ORC_E_INVALID;
  for (int64_t i = 0; i < n; i++) {
    const double layer[8] = {
        isnan(slope[i]) ? 0.0 : (double)slope[i],
        isnan(rough[i]) ? 0.0 : (double)rough[i],
        isnan(density[i]) ? 0.0 : (double)density[i],
        (flags[i] >> 1) & 1, (flags[i] >> 2) & 1, (flags[i] >> 3) & 1, (flags[i] >> 4) & 1,
        (flags[i] & 1) ? 0.0 : 1.0};
    double c = 0.0, a = 0.0;
    for (int k = 0; k < 8; k++) {
      c += w[k] * layer[k];
      a += fabs(w[k] * layer[k]);
    }
    cost[i] = c;
    mag[i] = a;
  }
  return ORC_OK;
}

int32_t orc_get_stats(const orc_map* m, orc_stats* out) {
  if (!m || !out) return ORC_E_INVALID;
  *out = m->st;
  return ORC_OK;
}

int32_t orc_get_origin(const orc_map* m, int32_t origin[3]) {
  if (!m || !origin) return ORC_E_INVALID;
  origin[0] = m->origin[0];
  origin[1] = m->origin[1];
  origin[2] = m->origin[2];
  return ORC_OK;
}
