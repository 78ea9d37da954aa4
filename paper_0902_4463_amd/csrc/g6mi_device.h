// Device-side building blocks shared by the single-system kernels
// (g6mi_kernels.hip) and the batched multi-cluster kernel (g6mi_batch.hip):
// the j-predictor of one record, the pair interaction in the three precision
// variants, the two-level float32 summation, and the per-lane state that
// walks LDS-staged j-tiles (two i-particles per lane, or one i-particle
// shared by L lanes).
#pragma once

#include "g6mi_internal.h"
#include "../../include/g6mi.h"

#include <cmath>
#include <cfloat>
#include <type_traits>

namespace g6mi {

// j-records per group: the unit of the nearest-neighbour bookkeeping, of the
// neighbour-list flags and of the first level of float32 summation.
constexpr int kGroup = G6MI_GROUP;
// Group length of the spatially ordered kernel (force_spatial).  Nine tiles
// in ten are far there, their pair terms within a small factor of each
// other, and the near tiles fold every group into float64; a longer group
// spreads the per-group work (nearest-neighbour and neighbour tests, the
// add into the tile sums) over more pairs.
constexpr int kSpatialGroup = G6MI_SPATIAL_GROUP;
static_assert(kTile / kGroup <= 32, "one mask bit per group");
static_assert(kTile % kGroup == 0, "whole groups per tile");
static_assert(kTile == kWG, "one j-record per lane when a tile is predicted in place");

// Predicted record size in float4 units.
template <int PREC> constexpr int rec4() {
  return PREC == G6MI_PREC_DS ? 3 : (PREC == G6MI_PREC_FP32 ? 2 : 4);
}

template <int PREC> using real_t = std::conditional_t<PREC == G6MI_PREC_FP64, double, float>;

// ---------------------------------------------------------------- predictor

// The float64 j-memory entries of one slot that the predictor reads: a
// kernel can load the next tile's entries into registers while it works on
// the current one, and predict them later.
struct JRaw {
  double t, m, x[3], v[3], a2[3], j6[3];
  __device__ __forceinline__ void load(const JMem &jm, size_t k) {
    t = jm.t[k];
    m = jm.m[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const size_t e = d * jm.cap + k;
      x[d] = jm.x[e];
      v[d] = jm.v[e];
      a2[d] = jm.a2[e];
      j6[d] = jm.j6[e];
    }
  }
};

// Sec. 2.2, Eq. (1) and (2), with the stored coefficients a2 = a/2 and
// j6 = jerk/6 and tau = t_i - t_j, evaluated by Horner's rule in float64.
// The double-single split (Sec. 2.2, Bailey's format) is hi = fl32(x),
// lo = fl32(x - hi); x - hi is exact in float64.  Writes the record of the
// slot held in r in the layout of the precision variant to o (global memory
// or LDS).
template <int PREC>
__device__ __forceinline__ void predict_raw(const JRaw &r, double ti, float4 *__restrict__ o) {
  const double tau = ti - r.t;
  double xp[3], vp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double c2 = r.a2[d], c3 = r.j6[d], c1 = r.v[d];
    xp[d] = r.x[d] + tau * (c1 + tau * (c2 + tau * c3));
    vp[d] = c1 + tau * (2.0 * c2 + tau * (3.0 * c3));
  }
  const double mk = r.m;
  if constexpr (PREC == G6MI_PREC_DS) {
    float hi[3], lo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      hi[d] = static_cast<float>(xp[d]);
      lo[d] = static_cast<float>(xp[d] - static_cast<double>(hi[d]));
    }
    o[0] = make_float4(hi[0], hi[1], hi[2], static_cast<float>(mk));
    o[1] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    o[2] = make_float4(static_cast<float>(vp[0]), static_cast<float>(vp[1]),
                       static_cast<float>(vp[2]), 0.0f);
  } else if constexpr (PREC == G6MI_PREC_FP32) {
    o[0] = make_float4(static_cast<float>(xp[0]), static_cast<float>(xp[1]),
                       static_cast<float>(xp[2]), static_cast<float>(mk));
    o[1] = make_float4(static_cast<float>(vp[0]), static_cast<float>(vp[1]),
                       static_cast<float>(vp[2]), 0.0f);
  } else {
    double2 *o2 = reinterpret_cast<double2 *>(o);
    o2[0] = make_double2(xp[0], xp[1]);
    o2[1] = make_double2(xp[2], mk);
    o2[2] = make_double2(vp[0], vp[1]);
    o2[3] = make_double2(vp[2], 0.0);
  }
}

// The record of slot k predicted to ti (predict_raw on its j-memory entries).
template <int PREC>
__device__ __forceinline__ void predict_record(const JMem &jm, size_t k, double ti,
                                               float4 *__restrict__ o) {
  JRaw r;
  r.load(jm, k);
  predict_raw<PREC>(r, ti, o);
}

// ------------------------------------------------------------- interaction

// 1/sqrt(s) in float64: the hardware estimate refined by Newton-Raphson
// steps, y <- y + y (1 - s y^2) / 2, each roughly doubling the correct bits.
// One step leaves about 1e-14 relative in 1/r (force errors against the
// oracle 9e-15 on a Plummer sphere of 1024 with eps = 1/64 and 2e-13 with
// hard binaries at eps = 0, against 5e-15 and 2e-13 with two steps), and
// the float64 kernel runs 11% faster.
__device__ __forceinline__ double rsqrt_f64(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < G6MI_RSQ64_STEPS; ++it) {
    const double e = fma(-s * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Per-lane position and velocity of one i-particle.
template <int PREC> struct IState;

template <> struct IState<G6MI_PREC_DS> {
  float xh[3], xl[3], v[3];
};
template <> struct IState<G6MI_PREC_FP32> {
  float x[3], v[3];
};
template <> struct IState<G6MI_PREC_FP64> {
  double x[3], v[3];
};

// Running sums of one i-particle's pair terms: acceleration, the two jerk
// parts (m w / r^3 and m (r.w) r / r^5) and m / r.
//
// Float32 variants sum in two levels before the float64 totals: a fresh
// group of kGroup pairs, then the group sums into the tile sums.  A close
// neighbour's term can exceed the far-field terms by 10^4 or more; added one
// by one to a partial sum holding it, terms below half its ulp would round
// away entirely, a systematic loss up to ~1e-5.  Within a group at most
// kGroup - 1 terms meet such a partial, and group sums are large enough to
// round rather than vanish.
template <class R> struct Sums {
  R a[3], j1[3], j2[3], p;
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] = j1[k] = j2[k] = R(0);
    p = R(0);
  }
  __device__ __forceinline__ void add(const Sums &o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a[k] += o.a[k];
      j1[k] += o.j1[k];
      j2[k] += o.j2[k];
    }
    p += o.p;
  }
};

// Separation of i and one j-record: r = x_j - x_i (Eq. (3) for DS), the
// velocity difference and r^2 without softening.
template <int PREC>
__device__ __forceinline__ void separation(const IState<PREC> &st, const float4 *__restrict__ rec,
                                           real_t<PREC> d[3], real_t<PREC> w[3], real_t<PREC> &mj) {
  if constexpr (PREC == G6MI_PREC_DS) {
    const float4 p = rec[0], q = rec[1], v = rec[2];
    d[0] = (p.x - st.xh[0]) + (q.x - st.xl[0]);
    d[1] = (p.y - st.xh[1]) + (q.y - st.xl[1]);
    d[2] = (p.z - st.xh[2]) + (q.z - st.xl[2]);
    w[0] = v.x - st.v[0];
    w[1] = v.y - st.v[1];
    w[2] = v.z - st.v[2];
    mj = p.w;
  } else if constexpr (PREC == G6MI_PREC_FP32) {
    const float4 p = rec[0], v = rec[1];
    d[0] = p.x - st.x[0];
    d[1] = p.y - st.x[1];
    d[2] = p.z - st.x[2];
    w[0] = v.x - st.v[0];
    w[1] = v.y - st.v[1];
    w[2] = v.z - st.v[2];
    mj = p.w;
  } else {
    const double2 *r2 = reinterpret_cast<const double2 *>(rec);
    const double2 p0 = r2[0], p1 = r2[1], w0 = r2[2], w1 = r2[3];
    d[0] = p0.x - st.x[0];
    d[1] = p0.y - st.x[1];
    d[2] = p1.x - st.x[2];
    w[0] = w0.x - st.v[0];
    w[1] = w0.y - st.v[1];
    w[2] = w1.x - st.v[2];
    mj = p1.y;
  }
}

// r^2 in one fixed expression, so that every path takes the same neighbour
// decisions for the same pair
template <int PREC>
__device__ __forceinline__ real_t<PREC> sq3(const real_t<PREC> d[3]) {
  return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

template <int PREC>
__device__ __forceinline__ real_t<PREC> r2_of(const IState<PREC> &st, const float4 *__restrict__ rec) {
  real_t<PREC> d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  return sq3<PREC>(d);
}

// One pair (i, j).  MASK: compare the j-slot with the i-particle's own slot
// and drop the self pair.  NBL: build neighbour lists.
template <int PREC, bool MASK, bool NBL>
__device__ __forceinline__ void pair(const IState<PREC> &st, Sums<real_t<PREC>> &acc,
                                     const float4 *__restrict__ rec,
                                     int jslot, int islot, real_t<PREC> eps2,
                                     real_t<PREC> h2, real_t<PREC> &best, int &bslot,
                                     int *__restrict__ nb_count, int *__restrict__ nb_row) {
  using R = real_t<PREC>;
  R d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  const R dx = d[0], dy = d[1], dz = d[2], dvx = w[0], dvy = w[1], dvz = w[2];
  R r2u = sq3<PREC>(d);
  R s = r2u + eps2;
  if constexpr (MASK) {
    const bool self = (jslot == islot);
    mj = self ? R(0) : mj;
    s = self ? R(1) : s;
    r2u = self ? R(INFINITY) : r2u;
  }
  R rinv;
  if constexpr (PREC == G6MI_PREC_FP64) rinv = rsqrt_f64(s);
  else rinv = __builtin_amdgcn_rsqf(s);
  const R rinv2 = rinv * rinv;
  const R mr = mj * rinv;          // m / r
  const R mr3 = mr * rinv2;        // m / r^3
  const R rv = dx * dvx + dy * dvy + dz * dvz;
  const R mr3t = mr3 * (rv * rinv2); // m (r.v) / r^5
  acc.p += mr;
  acc.a[0] += mr3 * dx;
  acc.a[1] += mr3 * dy;
  acc.a[2] += mr3 * dz;
  acc.j1[0] += mr3 * dvx;
  acc.j1[1] += mr3 * dvy;
  acc.j1[2] += mr3 * dvz;
  acc.j2[0] += mr3t * dx;
  acc.j2[1] += mr3t * dy;
  acc.j2[2] += mr3t * dz;
  if (r2u < best) { // strict: the first (lowest) slot wins a tie
    best = r2u;
    bslot = jslot;
  }
  if constexpr (NBL) {
    if (r2u < h2) {
      const int pos = atomicAdd(nb_count, 1);
      if (pos < kNbMax) nb_row[pos] = jslot;
    }
  }
}

// The pair terms of Sec. 2.3 added to `acc`; returns the softened r^2 + eps2
// for the neighbour search of the grouped paths: a group's minimum of it
// picks the group that the exact search re-examines (resolve_group, with
// r2_of), and is compared with nb_flag_bound(h2, eps2) to flag groups that
// may hold neighbours.  Forming it with eps2 as the first addend takes one
// operation fewer per pair than r^2 and then r^2 + eps2; with eps2 = 0 it
// has the bits of sq3.  No self test: the caller only uses it on tiles that
// hold no i-particle's own slot.  FIRST: the group's first pair sets the
// sums instead of adding to them.
// SELF: the pair is the i-particle with its own record when `self`; its
// inverse distance is taken as zero (every term then adds an exact zero,
// also at eps2 = 0) and its r^2 as +inf, so that it is neither a nearest
// neighbour nor a neighbour.
template <int PREC, bool FIRST = false, bool SELF = false>
__device__ __forceinline__ real_t<PREC> pair_core(const IState<PREC> &st, Sums<real_t<PREC>> &acc,
                                                  const float4 *__restrict__ rec, real_t<PREC> eps2,
                                                  bool self = false) {
  using R = real_t<PREC>;
  R d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  R s = fma(d[2], d[2], fma(d[1], d[1], fma(d[0], d[0], eps2)));
  constexpr bool kInfSelf = SELF && PREC != G6MI_PREC_FP64 && G6MI_SELF_INF;
  // float32: the self pair's r^2 becomes +inf, and the hardware's
  // 1/sqrt(+inf) is +0, so one select serves both uses (float64's Newton
  // steps would turn +inf * 0 into NaN, so it selects rinv instead)
  if constexpr (kInfSelf) s = self ? R(INFINITY) : s;
  R rinv;
  if constexpr (PREC == G6MI_PREC_FP64) rinv = rsqrt_f64(s);
  else rinv = __builtin_amdgcn_rsqf(s);
  if constexpr (SELF && !kInfSelf) rinv = self ? R(0) : rinv;
  const R rinv2 = rinv * rinv;
  const R mr = mj * rinv;
  const R mr3 = mr * rinv2;
  const R rv = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
  const R mr3t = mr3 * (rv * rinv2);
  if constexpr (FIRST) {
    acc.p = mr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      acc.a[k] = mr3 * d[k];
      acc.j1[k] = mr3 * w[k];
      acc.j2[k] = mr3t * d[k];
    }
  } else {
    acc.p += mr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      acc.a[k] += mr3 * d[k];
      acc.j1[k] += mr3 * w[k];
      acc.j2[k] += mr3t * d[k];
    }
  }
  if constexpr (SELF && !kInfSelf) return self ? R(INFINITY) : s;
  else return s;
}

// Bound for the group neighbour flags, which compare the softened r^2 of
// pair_core: every pair with r2_of(...) < h2 has a softened r^2 below it,
// whatever the rounding of the two (each is three rounded operations, some
// float32 units of the last place; the factor is 16 of them).  A flag only
// selects a group for the exact test.
template <class R> __device__ __forceinline__ R nb_flag_bound(R h2, R eps2) {
  return (h2 + eps2) * R(1.0 + 0x1p-20);
}

// i-particle `row` of the i-arrays in a's layout.  An invalid row (a padding
// lane) gets the origin, no own slot and h2 = -inf (no neighbours); its
// results are never stored.
template <int PREC>
__device__ __forceinline__ void load_i(IState<PREC> &st, const ForceArgs &a, int row, bool valid,
                                       int &islot, real_t<PREC> &h2) {
  using R = real_t<PREC>;
  double xi[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0};
  islot = -1;
  h2 = R(-INFINITY);
  if (valid) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xi[d] = a.xi[3 * static_cast<size_t>(row) + d];
      vi[d] = a.vi[3 * static_cast<size_t>(row) + d];
    }
    islot = a.islot[row];
    h2 = static_cast<R>(a.h2[row]);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (PREC == G6MI_PREC_DS) {
      st.xh[d] = static_cast<float>(xi[d]);
      st.xl[d] = static_cast<float>(xi[d] - static_cast<double>(st.xh[d]));
      st.v[d] = static_cast<float>(vi[d]);
    } else {
      st.x[d] = static_cast<R>(xi[d]);
      st.v[d] = static_cast<R>(vi[d]);
    }
  }
}

// Float64 running totals of one i-particle: the tile sums are folded in
// after every tile (float32 variants sum at most kTile terms in float32).
struct Totals {
  double acc[3], jrk[3], pot;
};

template <class R>
__device__ __forceinline__ void fold(Sums<R> &ts, Totals &t) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    t.acc[d] += static_cast<double>(ts.a[d]);
    t.jrk[d] += static_cast<double>(ts.j1[d]) - 3.0 * static_cast<double>(ts.j2[d]);
  }
  t.pot += static_cast<double>(ts.p);
  ts.zero();
}

// Group sums g into the float32 tile sums ts, or straight into the float64
// totals t when `close` (the group holds a new nearest neighbour).  A close
// neighbour's terms can exceed the whole force several times over where the
// rest cancels them; in a float32 tile sum every later group would then
// round against that large partial (a particle of conditioning 10 in a long
// run lost 2e-6 of its acceleration so).  New nearest neighbours come rarely
// after the first few groups, so the float64 path is seldom taken.  Used by
// the narrow blocks (one i-particle per lane, registers to spare); in the
// two-per-lane kernels the branch's registers spill.
template <class R>
__device__ __forceinline__ void fold_or_add(Sums<R> &g, Sums<R> &ts, Totals &t, bool close) {
  if (close) fold(g, t);
  else ts.add(g);
}

// Per-pair path for tiles holding an own slot or the ragged end: the pair
// terms go through group sums of kGroup pairs (float32 variants) before the
// tile sums, as on the grouped path.  FOLD: each full group goes straight
// into the float64 totals instead (see WideLanes::tile); RECORD: a group that
// brought a new nearest neighbour does (fold_or_add).
template <int PREC, bool NBL, bool FOLD = false, bool RECORD = false>
struct MaskedRun {
  using R = real_t<PREC>;
  Sums<R> g;
  int n = 0;
  R best0 = R(INFINITY); // RECORD: the nearest-neighbour distance when the group began
  __device__ __forceinline__ void start() {
    g.zero();
    n = 0;
  }
  __device__ __forceinline__ void step(const IState<PREC> &st, Sums<R> &ts, Totals &tot, const float4 *rec,
                                       int jslot, int islot, R eps2, R h2, R &best, int &bslot, int *nb_count,
                                       int *nb_row) {
    if constexpr (PREC == G6MI_PREC_FP64) {
      pair<PREC, true, NBL>(st, ts, rec, jslot, islot, eps2, h2, best, bslot, nb_count, nb_row);
    } else {
      if constexpr (RECORD)
        if (n == 0) best0 = best;
      pair<PREC, true, NBL>(st, g, rec, jslot, islot, eps2, h2, best, bslot, nb_count, nb_row);
      if (++n == kGroup) {
        if constexpr (FOLD) fold(g, tot);
        else if constexpr (RECORD) fold_or_add(g, ts, tot, best < best0);
        else ts.add(g);
        start();
      }
    }
  }
  __device__ __forceinline__ void finish(Sums<R> &ts) {
    if constexpr (PREC != G6MI_PREC_FP64) ts.add(g);
  }
};

__device__ __forceinline__ void nb_append(int *__restrict__ nb_count, int *__restrict__ nb_slot,
                                          int row, int jslot) {
  const int pos = atomicAdd(nb_count + row, 1);
  if (pos < kNbMax) nb_slot[static_cast<size_t>(row) * kNbMax + pos] = jslot;
}

// j-slot of a record in the spatially sorted order (held in its second
// float4's w component; the first three floats are DS lo or velocity).
__device__ __forceinline__ int rec_slot(const float4 *rec) { return __float_as_int(rec[1].w); }

// Exact slot of a grouped-path nearest neighbour: re-examine the G records
// of the group starting at position grp (positions grp, grp +
// stride, ...) and merge the lexicographic (r^2, slot) minimum into (best,
// bslot).  The record at position js is at src + (js - base) records; its
// slot is js, or (SORTED) the slot stored in the record.  Clears grp.
template <int PREC, bool SORTED = false, int G = kGroup>
__device__ __forceinline__ void resolve_group(const IState<PREC> &st, int &grp, int stride,
                                              const float4 *__restrict__ src, int base,
                                              real_t<PREC> &best, int &bslot, int islot = -1) {
  constexpr int REC = rec4<PREC>();
  if (grp < 0) return;
  for (int u = 0; u < G; ++u) {
    const int js = grp + u * stride;
    const float4 *rec = src + static_cast<size_t>(js - base) * REC;
    const real_t<PREC> r = r2_of<PREC>(st, rec);
    const int sl = SORTED ? rec_slot(rec) : js;
    if (sl == islot) continue; // a group of a self tile (grouped path with SELF)
    if (r < best || (r == best && sl < bslot)) {
      best = r;
      bslot = sl;
    }
  }
  grp = -1;
}

// ------------------------------------------- two i-particles per lane

// Lane state of a wide block: every lane owns two i-particles (rows row0 and
// row1 of the i-arrays) and every lane of a wave reads the same j-record
// from LDS (a broadcast), so one LDS record serves 128 pairs.
//
// The j-loop runs in groups of kGroup records.  Nearest neighbour: one
// min() per pair; once per group the group minimum is compared with the
// running best and the group's first slot remembered (grp); the exact slot
// is recovered by re-examining that one group (resolve), where the first
// minimum wins as in a sequential scan.  The group minima are of the
// softened r^2 + eps2 (pair_core), monotone in r^2.  Neighbour lists need no
// per-pair test: a group may hold a neighbour of i only when its minimum is
// below nb_flag_bound(h_i^2, eps2), and only such groups are re-examined
// with the exact test.  Ragged tiles take the
// per-pair path; tiles that contain an i-particle's own slot take it too, or
// with SELFG the grouped path with the self pair excluded per pair.
//
// SORTED: the j-records are in a spatial order (positions are not slots):
// own-tile detection uses the own record's position (pos0, pos1, set by the
// caller), and the slots of neighbours and nearest neighbours are read from
// the records.  tile_far walks a far tile in float32 coordinates relative to
// the tile's centre (see force_spatial).
template <int PREC, bool NBL, bool SORTED = false, int G = kGroup>
struct WideLanes {
  static_assert(kTile % G == 0 && kTile / G <= 32, "whole groups per tile, one mask bit each");
  using R = real_t<PREC>;
  static constexpr int REC = rec4<PREC>();
  IState<PREC> s0, s1;
  int row0, row1, slot0, slot1, pos0, pos1;
  bool v0, v1;
  R h20, h21;
  Totals t0, t1;
  Sums<R> ts0, ts1; // tile sums
  // nearest neighbour: fast-path best r^2 and its group; exact best
  R gbest0, gbest1, ebest0, ebest1;
  int grp0, grp1, eslot0, eslot1;

  __device__ __forceinline__ void init(const ForceArgs &a, int r0, int r1, bool ok0, bool ok1) {
    row0 = r0;
    row1 = r1;
    v0 = ok0;
    v1 = ok1;
    load_i<PREC>(s0, a, r0, ok0, slot0, h20);
    load_i<PREC>(s1, a, r1, ok1, slot1, h21);
    pos0 = slot0;
    pos1 = slot1;
    t0 = Totals{{0, 0, 0}, {0, 0, 0}, 0};
    t1 = Totals{{0, 0, 0}, {0, 0, 0}, 0};
    ts0.zero();
    ts1.zero();
    gbest0 = gbest1 = ebest0 = ebest1 = R(INFINITY);
    grp0 = grp1 = eslot0 = eslot1 = -1;
  }

  // slot of the record at position jbase + jj, staged at tl
  __device__ __forceinline__ int jslot_at(const float4 *__restrict__ tl, int jbase, int jj) const {
    if constexpr (SORTED) return rec_slot(tl + jj * REC);
    else return jbase + jj;
  }

  // The cnt records at positions jbase .. jbase + cnt - 1 staged at tl.
  // FOLD: the float32 group sums go straight into the float64 totals, with
  // no float32 tile level.  Large terms of both signs from close neighbours
  // would otherwise cancel in one float32 tile sum, and every later group
  // would round against them.  The spatial kernel folds its near tiles; the
  // unordered DS kernels fold every tile (a particle of conditioning 9.5 in
  // a long run lost 2.1e-6 of its acceleration in the tile sum; folding cost
  // about 2.5% there).  Unlike fold_or_add it needs no branch, whose
  // registers spill heavily in these two-per-lane kernels.
  //
  // SELFG (unsorted records only): a full tile holding an own slot takes the
  // grouped path with the self pair excluded per pair (pair_core's SELF)
  // instead of the per-pair path.  Where the i-particles are a random subset
  // of the j-particles (block steps, batches of small clusters) nearly every
  // tile holds some lane's own slot.
  template <bool FOLD = false, bool SELFG = false>
  __device__ __forceinline__ void tile(const float4 *__restrict__ tl, int jbase, int cnt, R eps2,
                                       int *__restrict__ nb_count, int *__restrict__ nb_slot) {
    static_assert(!(SELFG && SORTED), "own records are found by slot");
    const bool self_here =
        (pos0 >= jbase && pos0 < jbase + cnt) || (pos1 >= jbase && pos1 < jbase + cnt);
    if (cnt < kTile || (!SELFG && __any(self_here))) {
      MaskedRun<PREC, NBL, FOLD> r0, r1;
      r0.start();
      r1.start();
      int *c0 = nb_count + (v0 ? row0 : 0), *c1 = nb_count + (v1 ? row1 : 0);
      int *l0 = nb_slot + static_cast<size_t>(v0 ? row0 : 0) * kNbMax;
      int *l1 = nb_slot + static_cast<size_t>(v1 ? row1 : 0) * kNbMax;
      for (int jj = 0; jj < cnt; ++jj) {
        const int js = jslot_at(tl, jbase, jj);
        r0.step(s0, ts0, t0, tl + jj * REC, js, slot0, eps2, h20, ebest0, eslot0, c0, l0);
        r1.step(s1, ts1, t1, tl + jj * REC, js, slot1, eps2, h21, ebest1, eslot1, c1, l1);
      }
      r0.finish(ts0);
      r1.finish(ts1);
    } else if (SELFG && __any(self_here)) {
      grouped<FOLD, true>(tl, jbase, eps2, nb_count, nb_slot);
    } else {
      grouped<FOLD, false>(tl, jbase, eps2, nb_count, nb_slot);
    }
    fold(ts0, t0);
    fold(ts1, t1);
  }

  // The grouped path of `tile` over a full tile; SELF: the pair of an
  // i-particle with its own slot adds zeros and is no (nearest) neighbour.
  template <bool FOLD, bool SELF>
  __device__ __forceinline__ void grouped(const float4 *__restrict__ tl, int jbase, R eps2,
                                          int *__restrict__ nb_count, int *__restrict__ nb_slot) {
    // own slots relative to the tile (outside 0 .. kTile - 1 when elsewhere)
    const int o0 = slot0 - jbase, o1 = slot1 - jbase;
    // bit k of nbm0 / nbm1: group k may hold a neighbour of i0 / i1
    unsigned nbm0 = 0u, nbm1 = 0u;
    const R f0 = nb_flag_bound(h20, eps2), f1 = nb_flag_bound(h21, eps2);
#pragma unroll G6MI_GROUP_UNROLL
    for (int g = 0; g < kTile; g += G) {
      R m0 = R(INFINITY), m1 = R(INFINITY);
      if constexpr (PREC == G6MI_PREC_FP64) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const float4 *rec = tl + (g + u) * REC;
          m0 = fmin(m0, pair_core<PREC, false, SELF>(s0, ts0, rec, eps2, g + u == o0));
          m1 = fmin(m1, pair_core<PREC, false, SELF>(s1, ts1, rec, eps2, g + u == o1));
        }
      } else {
        Sums<R> g0, g1; // group sums, set by the group's first pair
        m0 = pair_core<PREC, true, SELF>(s0, g0, tl + g * REC, eps2, g == o0);
        m1 = pair_core<PREC, true, SELF>(s1, g1, tl + g * REC, eps2, g == o1);
#pragma unroll
        for (int u = 1; u < G; ++u) {
          const float4 *rec = tl + (g + u) * REC;
          m0 = fmin(m0, pair_core<PREC, false, SELF>(s0, g0, rec, eps2, g + u == o0));
          m1 = fmin(m1, pair_core<PREC, false, SELF>(s1, g1, rec, eps2, g + u == o1));
        }
        if constexpr (FOLD) {
          fold(g0, t0);
          fold(g1, t1);
        } else {
          ts0.add(g0);
          ts1.add(g1);
        }
      }
      if (m0 < gbest0) {
        gbest0 = m0;
        grp0 = jbase + g;
      }
      if (m1 < gbest1) {
        gbest1 = m1;
        grp1 = jbase + g;
      }
      if constexpr (NBL) {
        // the group minimum also tells whether any record may be a neighbour
        nbm0 |= (m0 < f0 ? 1u : 0u) << (g / G);
        nbm1 |= (m1 < f1 ? 1u : 0u) << (g / G);
      }
    }
    if constexpr (NBL) {
      // rare: append the neighbours of the flagged groups
      while (nbm0 | nbm1) {
        const int k = __builtin_ctz(nbm0 | nbm1);
        const unsigned bit = 1u << k;
        for (int u = 0; u < G; ++u) {
          const int jj = k * G + u;
          const float4 *rec = tl + jj * REC;
          if ((nbm0 & bit) && (!SELF || jj != o0) && r2_of<PREC>(s0, rec) < h20)
            nb_append(nb_count, nb_slot, row0, jslot_at(tl, jbase, jj));
          if ((nbm1 & bit) && (!SELF || jj != o1) && r2_of<PREC>(s1, rec) < h21)
            nb_append(nb_count, nb_slot, row1, jslot_at(tl, jbase, jj));
        }
        nbm0 &= ~bit;
        nbm1 &= ~bit;
      }
    }
  }

  // Resolve the pending groups from records at src (position js at js - base).
  __device__ __forceinline__ void resolve(const float4 *__restrict__ src, int base) {
    resolve_group<PREC, SORTED, G>(s0, grp0, 1, src, base, ebest0, eslot0, slot0);
    resolve_group<PREC, SORTED, G>(s1, grp1, 1, src, base, ebest1, eslot1, slot1);
  }

  // Spatially ordered records (src, n of them, in the order of the tiles):
  // start each particle's running group minimum at a strict upper bound of
  // its nearest-neighbour search's minimum, the softened r^2 to the record
  // next to its own (pos + 1, else pos - 1) times 1 + 2^-16, which covers
  // the few float32 units by which another path (the far separation) may
  // compute that pair, plus the least normal float32, which keeps the bound
  // above a pair at distance zero (eps2 = 0, coincident particles, where
  // both paths give exactly zero).  A split whose records hold nothing below
  // the bound then resolves no group and reports no candidate; the split
  // holding the nearest neighbour resolves it as before, since its group
  // minimum lies below the bound, so the merged nearest neighbour is
  // unchanged.  Far tiles farther than the bound need no neighbour work
  // (far_quiet).  A particle without its own record keeps +inf.
  __device__ __forceinline__ void seed_nn(const float4 *__restrict__ src, int n, R eps2) {
    static_assert(SORTED, "the record next to the own one is a near record only in a spatial order");
    auto bound = [&](const IState<PREC> &st, int pos, bool v) -> R {
      if (!v || pos < 0 || n < 2) return R(INFINITY);
      const int k = pos + 1 < n ? pos + 1 : pos - 1;
      R d[3], w[3], mj;
      separation<PREC>(st, src + static_cast<size_t>(k) * REC, d, w, mj);
      const R s = fma(d[2], d[2], fma(d[1], d[1], fma(d[0], d[0], eps2)));
      return fma(s, R(1.0 + 0x1p-16), R(0x1p-126));
    };
    gbest0 = bound(s0, pos0, v0);
    gbest1 = bound(s1, pos1, v1);
  }

  // Whether a far tile (every record within rt of the tile's centre, which
  // rt bounds from above; this lane's i-particles at f0, f1 relative to the
  // centre) can neither lower this lane's running group minimum of the
  // softened r^2 nor raise a neighbour flag: the least softened r^2 any of
  // its records can give, (|x_i - c| - rt)^2 + eps2, exceeds both.  The
  // factors 1 -+ 2^-18 keep the bound below every computed value: the far
  // separation and the squares are each within a few float32 units of the
  // last place (2^-24) of the exact ones.  Then the tile's group minima
  // would change nothing, and tile_far<false> gives the same results.
  // Padding lanes take no part.
  __device__ __forceinline__ bool far_quiet(const IState<G6MI_PREC_FP32> &f0, const IState<G6MI_PREC_FP32> &f1,
                                            float rt, R eps2) const {
    static_assert(PREC == G6MI_PREC_DS, "the far path refines the double-single variant");
    auto least = [&](const IState<G6MI_PREC_FP32> &f) {
      const float dc = sqrtf(fmaf(f.x[2], f.x[2], fmaf(f.x[1], f.x[1], f.x[0] * f.x[0])));
      const float gap = fmaxf(dc * (1.0f - 0x1p-18f) - rt * (1.0f + 0x1p-18f), 0.0f);
      return fmaf(gap, gap, eps2) * (1.0f - 0x1p-18f);
    };
    R need0 = gbest0, need1 = gbest1;
    if constexpr (NBL) {
      need0 = fmaxf(need0, nb_flag_bound(h20, eps2));
      need1 = fmaxf(need1, nb_flag_bound(h21, eps2));
    }
    return (!v0 || least(f0) > need0) && (!v1 || least(f1) > need1);
  }

  // A full far tile in float32 records relative to the tile's centre
  // (float4{x - c, m}, float4{v, slot}) with the i-particles' positions
  // relative to the same centre in f0, f1 (their velocities as in s0, s1):
  // the grouped path of `tile` with a three-operation separation.  Nearest-
  // neighbour groups are kept by position, as on the DS path.
  // NN = false: the tile cannot move this lane's nearest-neighbour search or
  // flag a neighbour (far_quiet), and the pairs add their terms alone; the
  // sums are those of NN = true.
  template <bool NN = true>
  __device__ __forceinline__ void tile_far(const float4 *__restrict__ ftl, int jbase, R eps2,
                                           const IState<G6MI_PREC_FP32> &f0, const IState<G6MI_PREC_FP32> &f1,
                                           int *__restrict__ nb_count, int *__restrict__ nb_slot) {
    static_assert(PREC == G6MI_PREC_DS, "the far path refines the double-single variant");
    constexpr int FREC = rec4<G6MI_PREC_FP32>();
    unsigned nbm0 = 0u, nbm1 = 0u;
    const R b0 = nb_flag_bound(h20, eps2), b1 = nb_flag_bound(h21, eps2);
#pragma unroll G6MI_GROUP_UNROLL
    for (int g = 0; g < kTile; g += G) {
      Sums<R> g0, g1;
      R m0 = pair_core<G6MI_PREC_FP32, true>(f0, g0, ftl + g * FREC, eps2);
      R m1 = pair_core<G6MI_PREC_FP32, true>(f1, g1, ftl + g * FREC, eps2);
#pragma unroll
      for (int u = 1; u < G; ++u) {
        const float4 *rec = ftl + (g + u) * FREC;
        const R q0 = pair_core<G6MI_PREC_FP32>(f0, g0, rec, eps2);
        const R q1 = pair_core<G6MI_PREC_FP32>(f1, g1, rec, eps2);
        if constexpr (NN) {
          m0 = fmin(m0, q0);
          m1 = fmin(m1, q1);
        }
      }
      ts0.add(g0);
      ts1.add(g1);
      if constexpr (NN) {
        if (m0 < gbest0) {
          gbest0 = m0;
          grp0 = jbase + g;
        }
        if (m1 < gbest1) {
          gbest1 = m1;
          grp1 = jbase + g;
        }
        if constexpr (NBL) {
          nbm0 |= (m0 < b0 ? 1u : 0u) << (g / G);
          nbm1 |= (m1 < b1 ? 1u : 0u) << (g / G);
        }
      }
    }
    if constexpr (NN && NBL) {
      while (nbm0 | nbm1) {
        const int k = __builtin_ctz(nbm0 | nbm1);
        const unsigned bit = 1u << k;
        for (int u = 0; u < G; ++u) {
          const float4 *rec = ftl + (k * G + u) * FREC;
          if ((nbm0 & bit) && r2_of<G6MI_PREC_FP32>(f0, rec) < h20) nb_append(nb_count, nb_slot, row0, rec_slot(rec));
          if ((nbm1 & bit) && r2_of<G6MI_PREC_FP32>(f1, rec) < h21) nb_append(nb_count, nb_slot, row1, rec_slot(rec));
        }
        nbm0 &= ~bit;
        nbm1 &= ~bit;
      }
    }
    fold(ts0, t0);
    fold(ts1, t1);
  }
};

// ------------------------------------- one i-particle on L lanes

// Lane state of a narrow block: ipw i-particles per workgroup (a power of
// two, at most kWG) and L = kWG / ipw lanes per i-particle.  Lane `sub` of an
// i-particle handles records sub, sub + L, sub + 2L, ... of every tile
// (Sec. 2.3, Fig. accMP1: spare threads split the j-range).  Full tiles
// without an own slot use the grouped path of WideLanes with stride-L
// groups.
template <int PREC, bool NBL>
struct NarrowLane {
  using R = real_t<PREC>;
  static constexpr int REC = rec4<PREC>();
  IState<PREC> st;
  int row, slot, sub, log2L, L, K;
  bool valid;
  R h2;
  Totals t;
  Sums<R> ts;
  R gbest, ebest;
  int grp, eslot;

  __device__ __forceinline__ void init(const ForceArgs &a, int r, bool ok, int sub_, int log2L_) {
    row = r;
    valid = ok;
    sub = sub_;
    log2L = log2L_;
    L = 1 << log2L_;
    K = kTile >> log2L_; // records per lane in a full tile
    load_i<PREC>(st, a, r, ok, slot, h2);
    t = Totals{{0, 0, 0}, {0, 0, 0}, 0};
    ts.zero();
    gbest = ebest = R(INFINITY);
    grp = eslot = -1;
  }

  // A full tile holding an own slot takes the grouped path with the self
  // pair excluded per pair (pair_core's SELF); ragged tiles and tiles of
  // fewer than kGroup records per lane take the per-pair path.
  __device__ __forceinline__ void tile(const float4 *__restrict__ tl, int jbase, int cnt, R eps2,
                                       int *__restrict__ nb_count, int *__restrict__ nb_slot) {
    const bool self_here = slot >= jbase && slot < jbase + cnt;
    if (cnt < kTile || K < kGroup) {
      int *nb_cnt = nb_count + (valid ? row : 0);
      int *nb_row = nb_slot + static_cast<size_t>(valid ? row : 0) * kNbMax;
      MaskedRun<PREC, NBL, false, true> run;
      run.start();
      for (int jj = sub; jj < cnt; jj += L)
        run.step(st, ts, t, tl + jj * REC, jbase + jj, slot, eps2, h2, ebest, eslot, nb_cnt, nb_row);
      run.finish(ts);
    } else if (__any(self_here)) {
      grouped<true>(tl, jbase, eps2, nb_count, nb_slot);
    } else {
      grouped<false>(tl, jbase, eps2, nb_count, nb_slot);
    }
    fold(ts, t);
  }

  template <bool SELF>
  __device__ __forceinline__ void grouped(const float4 *__restrict__ tl, int jbase, R eps2,
                                          int *__restrict__ nb_count, int *__restrict__ nb_slot) {
    const int o = slot - jbase; // own slot relative to the tile
    unsigned nbm = 0u;
    const R fb = nb_flag_bound(h2, eps2);
    for (int k0 = 0; k0 < K; k0 += kGroup) {
      R m = R(INFINITY);
      if constexpr (PREC == G6MI_PREC_FP64) {
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          const int jj = sub + ((k0 + u) << log2L);
          m = fmin(m, pair_core<PREC, false, SELF>(st, ts, tl + jj * REC, eps2, jj == o));
        }
      } else {
        Sums<R> gs; // group sums, set by the group's first pair
        m = pair_core<PREC, true, SELF>(st, gs, tl + (sub + (k0 << log2L)) * REC, eps2, sub + (k0 << log2L) == o);
#pragma unroll
        for (int u = 1; u < kGroup; ++u) {
          const int jj = sub + ((k0 + u) << log2L);
          m = fmin(m, pair_core<PREC, false, SELF>(st, gs, tl + jj * REC, eps2, jj == o));
        }
        if constexpr (G6MI_NARROW_FOLD) fold(gs, t);
        else fold_or_add(gs, ts, t, m < gbest);
      }
      if (m < gbest) {
        gbest = m;
        grp = jbase + sub + (k0 << log2L);
      }
      if constexpr (NBL) nbm |= (m < fb ? 1u : 0u) << (k0 / kGroup);
    }
    if constexpr (NBL) {
      while (nbm) { // rare: append the neighbours of the flagged groups
        const int g = __builtin_ctz(nbm);
        nbm &= nbm - 1u;
        for (int u = 0; u < kGroup; ++u) {
          const int jj = sub + ((g * kGroup + u) << log2L);
          if ((!SELF || jj != o) && r2_of<PREC>(st, tl + jj * REC) < h2) nb_append(nb_count, nb_slot, row, jbase + jj);
        }
      }
    }
  }

  __device__ __forceinline__ void resolve(const float4 *__restrict__ src, int base) {
    resolve_group<PREC>(st, grp, L, src, base, ebest, eslot, slot);
  }

  // Add the L lane totals of each i-particle in a fixed order.  The lanes of
  // i-particle il are tid = sub * ipw + il.  Within a wave (ipw < 64: 64 /
  // ipw of them per wave) they meet in an xor butterfly of cross-lane
  // exchanges over the lane bits from ipw up to 32; each exchange adds the
  // same two operands on both lanes, so all of them end with the same bits.
  // The P = 256 / max(ipw, 64) parts left (one per wave, or one per lane
  // when ipw >= 64) go through `red` (LDS, [9][kWG] doubles; the caller
  // synchronises before reusing it), and lane il adds parts 1 .. P - 1 in
  // order.  Afterwards the lanes with sub == 0 (tid = il) hold the
  // i-particle's totals in t and its nearest-neighbour candidate in
  // (bestd, bslot).
  __device__ __forceinline__ void lane_sum(double *red, int tid, int il, int ipw, double &bestd,
                                           int &bslot) {
    bestd = static_cast<double>(ebest);
    bslot = eslot;
    if (L == 1) return;
    for (int m = ipw; m < 64; m <<= 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        t.acc[d] += __shfl_xor(t.acc[d], m);
        t.jrk[d] += __shfl_xor(t.jrk[d], m);
      }
      t.pot += __shfl_xor(t.pot, m);
      const double r2o = __shfl_xor(bestd, m);
      const int so = __shfl_xor(bslot, m);
      nn_merge_lane(r2o, so, bestd, bslot);
    }
    const int stride = ipw < 64 ? 64 : ipw; // lanes between the holders of two parts
    const int nparts = kWG / stride;
    if (nparts == 1) return;
    int *rslot = reinterpret_cast<int *>(red + 8 * kWG);
    __syncthreads();
    if (tid >= stride && (tid & (stride - 1)) == il) { // holder of part tid / stride > 0
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d * kWG + tid] = t.acc[d];
        red[(3 + d) * kWG + tid] = t.jrk[d];
      }
      red[6 * kWG + tid] = t.pot;
      red[7 * kWG + tid] = bestd;
      rslot[tid] = bslot;
    }
    __syncthreads();
    if (tid == il) {
      for (int p = 1; p < nparts; ++p) {
        const int o = p * stride + il;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          t.acc[d] += red[d * kWG + o];
          t.jrk[d] += red[(3 + d) * kWG + o];
        }
        t.pot += red[6 * kWG + o];
        nn_merge_lane(red[7 * kWG + o], rslot[o], bestd, bslot);
      }
    }
  }

  // (r2o, so) merged into (bestd, bslot): the lexicographic (r^2, slot)
  // minimum over valid slots (order-independent).
  __device__ __forceinline__ static void nn_merge_lane(double r2o, int so, double &bestd, int &bslot) {
    if (so >= 0 && (r2o < bestd || (r2o == bestd && (bslot < 0 || so < bslot)))) {
      bestd = r2o;
      bslot = so;
    }
  }
};

// LDS bytes of a narrow block: the tile, or the lane-sum area after it.
template <int PREC> constexpr int narrow_lds_bytes() {
  constexpr int red = kWG * 9 * 8; // 7 sums + r2 + slot per lane
  constexpr int tile = kTile * rec4<PREC>() * 16;
  return red > tile ? red : tile;
}

// Register budget: G6MI_WIDE_WAVES waves per SIMD for the float32
// variants; float64 state takes twice the registers, so one wave fewer.
template <int PREC> constexpr int wide_waves() {
  return G6MI_WIDE_WAVES <= 1 ? 1 : (PREC == G6MI_PREC_FP64 ? G6MI_WIDE_WAVES - 1 : G6MI_WIDE_WAVES);
}

// ------------------------------------------------------------ finalisation

// Nearest-neighbour candidate (r2, sl) merged into (best, bslot): the
// lexicographic (r^2, slot) minimum over valid slots, so the merge order
// does not matter.
__device__ __forceinline__ void nn_merge(double r2, int sl, double &best, int &bslot) {
  if (sl >= 0 && (r2 < best || (r2 == best && (bslot < 0 || sl < bslot)))) {
    best = r2;
    bslot = sl;
  }
}

// The nsplit j-split partials of one i-particle added by a group of G lanes
// (G a power of two up to 64) of one wave, every lane of the group active:
// lane g of the group sits xs lanes after lane g - 1 (split_lane_map puts
// the G lanes of an i-particle xs = 64 / G apart, so that the lanes with the
// same g read consecutive i-particles).  Component c of split q is at
// part[q * sstride + c * cstride]; the candidates at nn_r2[q * nstride],
// nn_slot[q * nstride].  Lane g adds splits g, g + G, g + 2G, ... in that
// order in float64, its loads issued kAhead splits ahead of the additions
// (latency, not bandwidth, bounds a long sum); the G lane sums then meet in
// a butterfly of xor exchanges.  Each exchange adds two equal pairs of
// operands in either order, so all lanes of the group end with the same
// bits, and the order of additions is fixed by nsplit and G alone.  G = 1
// is the plain sum in split order.
__device__ __forceinline__ void split_sum(int nsplit, int G, int g, int xs, const double *__restrict__ part,
                                          size_t sstride, size_t cstride, const double *__restrict__ nn_r2,
                                          const int *__restrict__ nn_slot, size_t nstride, double s[7],
                                          double &best, int &bslot) {
  constexpr int kAhead = 4;
#pragma unroll
  for (int c = 0; c < 7; ++c) s[c] = 0.0;
  best = INFINITY;
  bslot = -1;
  int q = g;
  for (; q + (kAhead - 1) * G < nsplit; q += kAhead * G) {
    double v[kAhead][7], r2[kAhead];
    int sl[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      const size_t k = static_cast<size_t>(q + u * G);
#pragma unroll
      for (int c = 0; c < 7; ++c) v[u][c] = part[k * sstride + c * cstride];
      r2[u] = nn_r2[k * nstride];
      sl[u] = nn_slot[k * nstride];
    }
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
#pragma unroll
      for (int c = 0; c < 7; ++c) s[c] += v[u][c];
      nn_merge(r2[u], sl[u], best, bslot);
    }
  }
  for (; q < nsplit; q += G) {
    const size_t k = static_cast<size_t>(q);
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += part[k * sstride + c * cstride];
    nn_merge(nn_r2[k * nstride], nn_slot[k * nstride], best, bslot);
  }
  for (int m = 1; m < G; m <<= 1) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += __shfl_xor(s[c], m * xs);
    const double ob = __shfl_xor(best, m * xs);
    const int os = __shfl_xor(bslot, m * xs);
    nn_merge(ob, os, best, bslot);
  }
}

// Final result of one i-particle from its summed partials s (acc xyz, jerk
// xyz, sum m/r) and nearest-neighbour candidate: outputs go to row `row`,
// and its neighbour list is turned from slots into particle indices sorted
// ascending.  An overflowed list is queued in ovf_list (and its tag in
// ovf_tag when given) for the exact pass, counted in
// status[kStatusOverflowCount].  Returns the status flags of the row
// (bit 0 non-finite output, bit 1 neighbour overflow).
// nb_work: the interaction kernel counted the row's neighbours there instead
// of in nb_count; the count is moved to nb_count and nb_work[row] cleared
// for the next calculation (so that no launch has to clear it first).
__device__ __forceinline__ int finish_out(const double s[7], double best, int bslot, int row,
                                          const int *__restrict__ jindex,
                                          int *__restrict__ nb_count, int *__restrict__ nb_slot,
                                          bool nbl, double *__restrict__ acc, double *__restrict__ jerk,
                                          double *__restrict__ pot, int *__restrict__ nnb,
                                          double *__restrict__ r2nn, int *__restrict__ status,
                                          int *__restrict__ ovf_list, int *__restrict__ ovf_tag, int tag,
                                          int *__restrict__ nb_work = nullptr) {
  const size_t i = static_cast<size_t>(row);
  bool finite = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    acc[3 * i + d] = s[d];
    jerk[3 * i + d] = s[3 + d];
    finite = finite && isfinite(s[d]) && isfinite(s[3 + d]);
  }
  pot[i] = -s[6];
  finite = finite && isfinite(s[6]);
  if (nnb) nnb[i] = bslot >= 0 ? jindex[bslot] : -1;
  if (r2nn) r2nn[i] = bslot >= 0 ? best : INFINITY;
  int fl = finite ? 0 : 1;
  if (!nbl && nb_work) nb_count[i] = 0; // no list: no count left from an earlier call
  if (nbl) {
    int cnt;
    if (nb_work) {
      cnt = nb_work[i];
      nb_work[i] = 0;
      nb_count[i] = cnt;
    } else {
      cnt = nb_count[i];
    }
    int *lst = nb_slot + i * kNbMax;
    if (cnt > kNbMax) { // kept set decided later by the exact pass
      fl |= 2;
      const int q = atomicAdd(status + kStatusOverflowCount, 1);
      ovf_list[q] = row;
      if (ovf_tag) ovf_tag[q] = tag;
      return fl;
    }
    for (int a = 0; a < cnt; ++a) lst[a] = jindex[lst[a]];
    for (int a = 1; a < cnt; ++a) { // insertion sort: lists are short
      const int key = lst[a];
      int b = a - 1;
      while (b >= 0 && lst[b] > key) {
        lst[b + 1] = lst[b];
        --b;
      }
      lst[b + 1] = key;
    }
  }
  return fl;
}

// Lanes per i-particle of a split sum: one for up to 8 splits, else about a
// quarter of the splits, at most a wave, and fewer where the i-particles
// alone give lanes enough (ni * G at most 2^17).
__host__ __device__ constexpr int split_lanes(int nsplit, long long ni) {
  int G = 1;
  if (nsplit > 8)
    while (G < 64 && 4 * (2 * G) <= nsplit && ni * (2 * G) <= (1LL << 17)) G <<= 1;
  return G;
}

// Lane l of a wave, in groups of G lanes per i-particle (G a power of two up
// to 64): the wave holds w = 64 / G consecutive i-particles, lane l serving
// i-particle l mod w as member g = l / w of its group; the members of a
// group sit w lanes apart.
__device__ __forceinline__ void split_lane_map(int lane, int G, int &ioff, int &g, int &xs) {
  xs = 64 / G;
  ioff = lane & (xs - 1);
  g = lane / xs;
}

// ---------------------------------------------- neighbour-list overflow

// Rebuild the list of one overflowed i-particle as the kNbMax smallest
// particle indices among its neighbours in slots jlo .. jhi - 1, ascending
// (the oracle's convention), and write its neighbour count to *cnt.  Called
// by a whole workgroup.  The neighbour test is the one of the interaction
// kernels (same separation and r^2 arithmetic on the same records, fetched
// by rec_of(js, scratch)); count and list both come from this pass, so they
// agree even where the interaction kernel's own test (on the spatial path, a
// float32 separation relative to a tile centre) decided a pair at the
// sphere's edge the other way.  A binary search on the index threshold T
// counts the neighbours with index below T (indices biased to unsigned
// order); then the kNbMax of them below the final T are collected and
// rank-sorted.
template <int PREC, class RecOf>
__device__ void exact_list(const IState<PREC> &st, int slot, real_t<PREC> h2, int jlo, int jhi,
                           const int *__restrict__ jindex, RecOf rec_of, int *__restrict__ lst,
                           int *__restrict__ cnt, unsigned &s_cnt, int *s_keep) {
  const int tid = threadIdx.x;
  auto below = [&](unsigned long long T, bool collect) -> unsigned {
    __syncthreads();
    if (tid == 0) s_cnt = 0u;
    __syncthreads();
    unsigned c = 0u;
    for (int js = jlo + tid; js < jhi; js += kWG) {
      const unsigned key = static_cast<unsigned>(jindex[js]) ^ 0x80000000u;
      float4 buf[4];
      if (js != slot && key < T && r2_of<PREC>(st, rec_of(js, buf)) < h2) {
        if (collect) {
          const unsigned p = atomicAdd(&s_cnt, 1u);
          if (p < static_cast<unsigned>(kNbMax)) s_keep[p] = jindex[js];
        } else {
          ++c;
        }
      }
    }
    if (!collect && c) atomicAdd(&s_cnt, c);
    __syncthreads();
    return s_cnt;
  };
  constexpr unsigned long long kAll = 1ull << 32;
  const unsigned total = below(kAll, false);
  // smallest T with at least kNbMax neighbours below it (all of them when
  // there are no more than kNbMax)
  unsigned long long lo = 0ull, hi = kAll;
  if (total > static_cast<unsigned>(kNbMax)) {
    while (hi - lo > 1ull) {
      const unsigned long long mid = (lo + hi) >> 1;
      if (below(mid, false) >= static_cast<unsigned>(kNbMax)) hi = mid;
      else lo = mid;
    }
  }
  const unsigned got = below(hi, true);
  const int n = got < static_cast<unsigned>(kNbMax) ? static_cast<int>(got) : kNbMax;
  if (tid < n) { // rank sort; equal values ranked by position
    const int v = s_keep[tid];
    int r = 0;
    for (int u = 0; u < n; ++u) r += (s_keep[u] < v) | ((s_keep[u] == v) & (u < tid));
    lst[r] = v;
  }
  if (tid == 0) *cnt = static_cast<int>(total);
  __syncthreads(); // s_keep is reused by the next i-particle
}

} // namespace g6mi
