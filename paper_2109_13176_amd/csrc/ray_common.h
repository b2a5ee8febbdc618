// Device helpers of the ray pass and the traversal: point
// transform and return, dominant axis, exact segment entry voxel and the
// exact integer voxel walk (Sec. III-C of arXiv 2109.13176).
#pragma once
#include <math.h>

#include "gvom_internal.h"

namespace gvom {
namespace {

__device__ __forceinline__ int32_t wrap_add(int32_t s, int32_t n) { return s >= n ? s - n : s; }

// Sums an int over the 64 lanes of the wave.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ int32_t mod_pos(int32_t v, int32_t n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// x[k] for a lane-varying axis k, by selects (an indexed private array
// would go to scratch memory).
__device__ __forceinline__ int32_t sel3(const int k, const int32_t x0, const int32_t x1,
                                        const int32_t x2) {
  return k == 0 ? x0 : (k == 1 ? x1 : x2);
}

__device__ __forceinline__ int dominant_axis(const int32_t n[3]) {
  return (n[1] > n[0]) ? (n[2] > n[1] ? 2 : 1) : (n[2] > n[0] ? 2 : 0);
}

// Transform of point i (in firing order) and its return: q = Q16 world
// coordinates.  When the return lies in the window, f.hit is set and f.e /
// f.ow / f.ob locate its voxel (storage index, occupancy word and bit); the
// caller records the hit (record_hit_*).  Returns true when the ray can be
// traversed.
struct PointFlags {
  bool nonfinite = false, outrange = false, hit = false, dhit = false;
  int32_t e = 0;
  int64_t ow = 0;
  unsigned long long ob = 0;
};

template <bool DISTINCT>
__device__ __forceinline__ bool point_pass(const InsertArgs& a, const int i, int32_t q[3],
                                           PointFlags& f) {
  q[0] = q[1] = q[2] = 0;
  if (i >= a.n) return false;
  int pidx = i;
  if (a.fw > 1) {
    const int b = i / a.azimuths;
    pidx = (i - b * a.azimuths) * a.fw + b;
  }
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  const float p0 = a.xyz[3 * pidx + 0];
  const float p1 = a.xyz[3 * pidx + 1];
  const float p2 = a.xyz[3 * pidx + 2];
  if (!(isfinite(p0) && isfinite(p1) && isfinite(p2))) {
    f.nonfinite = true;
    return false;
  }
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    float w = __builtin_fmaf(a.R[3 * k + 0], p0, a.t[k]);
    w = __builtin_fmaf(a.R[3 * k + 1], p1, w);
    w = __builtin_fmaf(a.R[3 * k + 2], p2, w);
    const float u = w * a.inv_r;
    const bool okk = isfinite(w) && fabsf(u) < 32768.0f;
    q[k] = okk ? (int32_t)floorf(u * 65536.0f) : 0;
    ok = ok && okk;
    const int64_t dd = (int64_t)q[k] - a.S[k];
    ok = ok && dd < (1 << 27) && -dd < (1 << 27);
  }
  if (!ok) {
    f.outrange = true;
    return false;
  }
  int32_t l[3];
  bool win = true;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    l[k] = (q[k] >> 16) - a.O[k];
    win = win && l[k] >= 0 && l[k] < dims[k];
  }
  if (win) {  // the return
    const int32_t ex = wrap_add(l[0] + a.d.ro[0], dims[0]);
    const int32_t ey = wrap_add(l[1] + a.d.ro[1], dims[1]);
    const int32_t ez = wrap_add(l[2] + a.d.ro[2], dims[2]);
    const int32_t col = ex * dims[1] + ey;
    const int32_t e = col_base(a.d, ex, ey) + (ez << 4);
    f.e = e;
    f.ow = (int64_t)col * a.d.W + (ez >> 6);
    f.ob = 1ull << (ez & 63);
    f.hit = true;
    if (DISTINCT) {
      const uint32_t bit = 1u << (e & 31);
      const uint32_t old = atomicOr(&a.touch[(uint32_t)e >> 5], bit);
      f.dhit = !(old & bit);
    }
  }
  return true;
}

// Recording a hit takes a count, a minimum and an or.  The minimum and the or
// only move one way, so a plain read that already satisfies the update makes
// that atomic unnecessary.  The reads are issued first (record_hit_issue) and
// the conditional atomics later (record_hit_finish), so their round trip can
// overlap other work of the caller; a stale read only costs a redundant
// atomic.
struct HitReads {
  int32_t mz = 0;
  unsigned long long ow = 0;
};

__device__ __forceinline__ HitReads record_hit_issue(const InsertArgs& a, const PointFlags& f) {
  HitReads r;
  if (f.hit) {
    r.mz = a.minqz[f.e];
    r.ow = a.occ[f.ow];
    atomicAdd(&a.hits[f.e], 1);
  }
  return r;
}

__device__ __forceinline__ void record_hit_finish(const InsertArgs& a, const PointFlags& f,
                                                  const HitReads& r, const int32_t qz) {
  if (f.hit) {
    if (qz < r.mz) atomicMin(&a.minqz[f.e], qz);
    if (!(r.ow & f.ob)) atomicOr(&a.occ[f.ow], f.ob);
  }
}

// Voxel at which the ray S -> q enters world cell c along axis dm (c is not
// the sensor's cell): see the traversal pass below for the tie rule.
//
// At that instant another axis k lies at X_k = (S_k |D| + s_k |D_k| num) / |D|
// (Q units; D = the dominant component, s_k the sign along k, num = the
// dominant-axis distance from the sensor to the cell's boundary), in cell
// floor(X_k / 2^16).  A float estimate of that quotient is within 0.02 of it
// (|S_k| < 2^31, the displacement along k is below 2^27, each float step
// rounds to 2^-24 relative), so its floor is off by at most one and one
// exact 64-bit remainder test each way settles it.  All three axes are
// computed without branches (dm varies across a wave) and the dominant one
// is replaced by c.
__device__ __forceinline__ void entry_voxel(const int32_t S[3], const int32_t sg[3],
                                            const int32_t ad[3], const int dm, const int32_t c,
                                            int32_t v[3]) {
  const int32_t Sd = sel3(dm, S[0], S[1], S[2]);
  const int32_t dd = sel3(dm, ad[0], ad[1], ad[2]);
  const int32_t sd = sel3(dm, sg[0], sg[1], sg[2]);
  // |num| < 2^28 (the ray spans fewer than 2^11 cells); formed from the
  // cell offset so that no intermediate overflows
  const int32_t off = c - (Sd >> 16);
  const int32_t num = sd > 0 ? (off << 16) - (Sd & 0xFFFF) : (Sd & 0xFFFF) - ((off + 1) << 16);
  const int64_t den = (int64_t)dd << 16;
  const float rden = __builtin_amdgcn_rcpf((float)dd * 65536.0f);
  const float fdd = (float)dd, fnum = (float)num;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const int32_t sad = sg[k] * ad[k];
    const int64_t x = (int64_t)S[k] * dd + (int64_t)num * sad;
    int64_t qe = (int64_t)floorf(__builtin_fmaf((float)S[k], fdd, fnum * (float)sad) * rden);
    int64_t r = x - ((qe * dd) << 16);
    if (r < 0) {
      qe -= 1;
      r += den;
    } else if (r >= den) {
      qe += 1;
      r -= den;
    }
    if (r == 0 && sd < 0 && sg[k] < 0) qe -= 1;
    v[k] = k == dm ? c : (int32_t)qe;
  }
}

// Exact traversal state of one segment: remaining steps to the end voxel and
// to the window edge per axis, and the crossing-time differences.
//
// E_ab = num_a |D_b| - num_b |D_a| (num = distance from the sensor to the
// next boundary along the axis, Q units) decides which axis crosses first.
// It only changes by multiples of 2^16 (|D| << 16 per step), so its low 16
// bits are fixed and f = floor(E / 2^16) carries the rest: E >= 0 iff
// f >= 0, and E <= 0 iff f <= c with c = -1 when the low bits are not zero,
// else 0.  While both axes still move, the next crossings lie within one
// cell of the current point, so |E| <= 2^16 max(|D_a|, |D_b|) < 2^43 and f
// fits in 32 bits (|D| < 2^27); f of a finished axis is never consulted.
struct Walk {
  int32_t rem[3], room[3], sg[3], ad[3];
  int32_t fxy, fxz, fyz;
  int32_t cxy, cxz, cyz;
};

__device__ __forceinline__ void split_e(int64_t e, int32_t& f, int32_t& c) {
  f = (int32_t)(e >> 16);
  c = (e & 0xFFFF) ? -1 : 0;
}

// Starts the walk at world voxel v (inside the window, local l).
__device__ __forceinline__ void walk_init(const InsertArgs& a, const int32_t q[3],
                                          const int32_t v[3], const int32_t l[3], Walk& w) {
  const int32_t dims[3] = {a.d.nx, a.d.ny, a.d.nz};
  int32_t num[3];  // |num| < 2^28: v lies on the ray, which spans fewer than 2^11 cells
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const int32_t ev = q[k] >> 16;
    const int32_t dq = q[k] - a.S[k];
    w.sg[k] = dq > 0 ? 1 : (dq < 0 ? -1 : 0);
    w.ad[k] = dq < 0 ? -dq : dq;
    w.rem[k] = ev > v[k] ? ev - v[k] : v[k] - ev;
    w.room[k] = w.sg[k] > 0 ? dims[k] - 1 - l[k] : l[k];
    const int32_t off = v[k] - (a.S[k] >> 16), fr = a.S[k] & 0xFFFF;
    num[k] = w.sg[k] > 0 ? ((off + 1) << 16) - fr : fr - (off << 16);
  }
  split_e((int64_t)num[0] * w.ad[1] - (int64_t)num[1] * w.ad[0], w.fxy, w.cxy);
  split_e((int64_t)num[0] * w.ad[2] - (int64_t)num[2] * w.ad[0], w.fxz, w.cxz);
  split_e((int64_t)num[1] * w.ad[2] - (int64_t)num[2] * w.ad[1], w.fyz, w.cyz);
}

// One step: the axes with the smallest crossing time move; when several
// share it, the axes moving up step first (the shared boundary belongs to
// the upper cell) and the axes moving down in the next step.  Sets mx/my/mz
// and returns whether a moving axis left the window.
__device__ __forceinline__ bool walk_step(Walk& w, bool& mx, bool& my, bool& mz) {
  const bool ax = w.rem[0] > 0, ay = w.rem[1] > 0, az = w.rem[2] > 0;
  const bool px = w.sg[0] > 0, py = w.sg[1] > 0, pz = w.sg[2] > 0;
  mx = ax & (!ay | (w.fxy <= w.cxy)) & (!az | (w.fxz <= w.cxz));
  my = ay & (!ax | (w.fxy >= 0)) & (!az | (w.fyz <= w.cyz));
  mz = az & (!ax | (w.fxz >= 0)) & (!ay | (w.fyz >= 0));
  const bool up = (mx & px) | (my & py) | (mz & pz);
  mx = mx & (!up | px);
  my = my & (!up | py);
  mz = mz & (!up | pz);
  const bool out = (mx & (w.room[0] == 0)) | (my & (w.room[1] == 0)) | (mz & (w.room[2] == 0));
  w.rem[0] -= mx;
  w.rem[1] -= my;
  w.rem[2] -= mz;
  w.room[0] -= mx;
  w.room[1] -= my;
  w.room[2] -= mz;
  // wrapping unsigned adds: f of an axis that no longer moves may drift
  w.fxy = (int32_t)((uint32_t)w.fxy + (mx ? (uint32_t)w.ad[1] : 0u) - (my ? (uint32_t)w.ad[0] : 0u));
  w.fxz = (int32_t)((uint32_t)w.fxz + (mx ? (uint32_t)w.ad[2] : 0u) - (mz ? (uint32_t)w.ad[0] : 0u));
  w.fyz = (int32_t)((uint32_t)w.fyz + (my ? (uint32_t)w.ad[2] : 0u) - (mz ? (uint32_t)w.ad[1] : 0u));
  return out;
}

// Budgeted stepping for the segmented traversal.  cnt[k] = moves left along
// axis k before it either reaches the end voxel's coordinate (the axis stops
// moving) or, when stop[k], makes the move that leaves the window or the
// segment (the walk ends before that voxel).  While the walk is on,
// cnt[k] > 0 iff the axis still has steps to the end voxel, so the axis
// choice is the one of walk_step.
__device__ __forceinline__ void budget_init(const Walk& w, const int dom, const int32_t seg_len,
                                            int32_t cnt[3], bool stop[3]) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    int32_t T = w.room[k] + 1;                   // the move that leaves the window
    if (k == dom && seg_len < T) T = seg_len;    // the move that leaves the segment
    stop[k] = w.rem[k] >= T;
    cnt[k] = stop[k] ? T : w.rem[k];
  }
}

// One step of walk_step's rule under the budgets; returns whether the walk
// ends (a stopping axis spent its budget).
__device__ __forceinline__ bool budget_step(Walk& w, int32_t cnt[3], const bool stop[3],
                                            const bool px, const bool py, const bool pz,
                                            bool& mx, bool& my, bool& mz) {
  const bool ax = cnt[0] > 0, ay = cnt[1] > 0, az = cnt[2] > 0;
  mx = ax & (!ay | (w.fxy <= w.cxy)) & (!az | (w.fxz <= w.cxz));
  my = ay & (!ax | (w.fxy >= 0)) & (!az | (w.fyz <= w.cyz));
  mz = az & (!ax | (w.fxz >= 0)) & (!ay | (w.fyz >= 0));
  const bool up = (mx & px) | (my & py) | (mz & pz);
  mx = mx & (!up | px);
  my = my & (!up | py);
  mz = mz & (!up | pz);
  cnt[0] -= mx;
  cnt[1] -= my;
  cnt[2] -= mz;
  const bool out = (mx & stop[0] & (cnt[0] == 0)) | (my & stop[1] & (cnt[1] == 0)) |
                   (mz & stop[2] & (cnt[2] == 0));
  w.fxy = (int32_t)((uint32_t)w.fxy + (mx ? (uint32_t)w.ad[1] : 0u) - (my ? (uint32_t)w.ad[0] : 0u));
  w.fxz = (int32_t)((uint32_t)w.fxz + (mx ? (uint32_t)w.ad[2] : 0u) - (mz ? (uint32_t)w.ad[0] : 0u));
  w.fyz = (int32_t)((uint32_t)w.fyz + (my ? (uint32_t)w.ad[2] : 0u) - (mz ? (uint32_t)w.ad[1] : 0u));
  return out;
}

// a * b + c on the 24-bit multiplier (operands below 2^24; b uniform across
// the wave, taken from a scalar register).  Written out because the compiler
// widens the plain expression into a 64-bit multiply-add when the result
// feeds an address.
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// col_base with 24-bit multiplies: brick coordinates < 2^11, nby <= 2048
// and 16 nz <= 2048 keep every operand within 24 bits, and the index is
// below 2^31 for every map the library accepts.
__device__ __forceinline__ int32_t col_base24(const Dims& d, int32_t sx, int32_t sy) {
  const uint32_t b = mad_u24((uint32_t)(sx >> 2), (uint32_t)d.nby, (uint32_t)(sy >> 2));
  return (int32_t)mad_u24(b, (uint32_t)d.nz << 4, (uint32_t)(((sy & 3) << 2) | (sx & 3)));
}

}  // namespace
}  // namespace gvom
