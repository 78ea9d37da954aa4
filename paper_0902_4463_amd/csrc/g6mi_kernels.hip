// gfx950 kernels of the direct-summation force evaluation.
//
//   predict_kernel  -- j-particle predictor, Eq. (1)-(2) of Sec. 2.2, in
//                      float64, writing the predicted j-records in the layout
//                      of the selected precision variant (HBM-bound).
//   force_kernel    -- the i x j interaction (Sec. 2.3): LDS-staged j-tiles,
//                      j-split across workgroups, several lanes per
//                      i-particle when the block is small, nearest neighbour
//                      and neighbour lists fused in the same loop (VALU-bound).
//   reduce_kernel   -- fixed-order float64 sum of the j-split partials, the
//                      nearest-neighbour minimum and the neighbour-list
//                      finalisation (slot -> particle index, ascending).
//
// The pair interaction is elementwise per (i, j) pair, not a contraction,
// so it runs on the vector ALUs; no matrix-core instructions are used.

#include "g6mi_internal.h"
#include "../../include/g6mi.h"

#include <cmath>
#include <cfloat>
#include <type_traits>

namespace g6mi {

// j-records per group: the unit of the nearest-neighbour bookkeeping, of the
// neighbour-list flags and of the first level of float32 summation.
constexpr int kGroup = G6MI_GROUP;
static_assert(kTile / kGroup <= 32, "one mask bit per group");
static_assert(kTile % kGroup == 0, "whole groups per tile");

size_t pred_record_bytes(int prec) {
  switch (prec) {
  case G6MI_PREC_FP32: return 32;
  case G6MI_PREC_DS: return 48;
  default: return 64;
  }
}

// ---------------------------------------------------------------- predictor

// Sec. 2.2, Eq. (1) and (2), with the stored coefficients a2 = a/2 and
// j6 = jerk/6 and tau = t_i - t_j, evaluated by Horner's rule in float64.
// The double-single split (Sec. 2.2, Bailey's format) is hi = fl32(x),
// lo = fl32(x - hi); x - hi is exact in float64.
template <int PREC>
__global__ __launch_bounds__(256) void predict_kernel(
    int nj, double ti, const double *__restrict__ t,
    const double *__restrict__ m, const double *__restrict__ x,
    const double *__restrict__ v, const double *__restrict__ a2,
    const double *__restrict__ j6, size_t cap, void *__restrict__ out,
    int *__restrict__ nb_count, int ni, int *__restrict__ status) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < ni) nb_count[k] = 0; // fresh neighbour counters for this call
  if (k < kStatusWords) status[k] = 0;
  if (k >= nj) return;
  const double tau = ti - t[k];
  double xp[3], vp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t e = d * cap + k;
    const double c2 = a2[e], c3 = j6[e], c1 = v[e];
    xp[d] = x[e] + tau * (c1 + tau * (c2 + tau * c3));
    vp[d] = c1 + tau * (2.0 * c2 + tau * (3.0 * c3));
  }
  const double mk = m[k];
  if constexpr (PREC == G6MI_PREC_DS) {
    float hi[3], lo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      hi[d] = static_cast<float>(xp[d]);
      lo[d] = static_cast<float>(xp[d] - static_cast<double>(hi[d]));
    }
    float4 *o = static_cast<float4 *>(out) + 3 * static_cast<size_t>(k);
    o[0] = make_float4(hi[0], hi[1], hi[2], static_cast<float>(mk));
    o[1] = make_float4(lo[0], lo[1], lo[2], 0.0f);
    o[2] = make_float4(static_cast<float>(vp[0]), static_cast<float>(vp[1]),
                       static_cast<float>(vp[2]), 0.0f);
  } else if constexpr (PREC == G6MI_PREC_FP32) {
    float4 *o = static_cast<float4 *>(out) + 2 * static_cast<size_t>(k);
    o[0] = make_float4(static_cast<float>(xp[0]), static_cast<float>(xp[1]),
                       static_cast<float>(xp[2]), static_cast<float>(mk));
    o[1] = make_float4(static_cast<float>(vp[0]), static_cast<float>(vp[1]),
                       static_cast<float>(vp[2]), 0.0f);
  } else {
    double2 *o = static_cast<double2 *>(out) + 4 * static_cast<size_t>(k);
    o[0] = make_double2(xp[0], xp[1]);
    o[1] = make_double2(xp[2], mk);
    o[2] = make_double2(vp[0], vp[1]);
    o[3] = make_double2(vp[2], 0.0);
  }
}

// ------------------------------------------------------------- interaction

// Record size in float4 units.
template <int PREC> constexpr int rec4() {
  return PREC == G6MI_PREC_DS ? 3 : (PREC == G6MI_PREC_FP32 ? 2 : 4);
}

// 1/sqrt(s) in float64: the hardware estimate refined by two Newton-Raphson
// steps, y <- y + y (1 - s y^2) / 2, each roughly doubling the correct bits.
__device__ __forceinline__ double rsqrt_f64(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
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

template <int PREC> using real_t = std::conditional_t<PREC == G6MI_PREC_FP64, double, float>;

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

// ------------------------------------------------- interaction, wide blocks

// The pair terms of Sec. 2.3 added to `acc`; returns r^2 (without
// softening) for the neighbour search.  No self test: the caller only uses
// it on tiles that hold neither i-particle's own slot.
template <int PREC, bool FIRST = false>
__device__ __forceinline__ real_t<PREC> pair_core(const IState<PREC> &st, Sums<real_t<PREC>> &acc,
                                                  const float4 *__restrict__ rec, real_t<PREC> eps2) {
  using R = real_t<PREC>;
  R d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  const R r2u = sq3<PREC>(d);
  const R s = r2u + eps2;
  R rinv;
  if constexpr (PREC == G6MI_PREC_FP64) rinv = rsqrt_f64(s);
  else rinv = __builtin_amdgcn_rsqf(s);
  const R rinv2 = rinv * rinv;
  const R mr = mj * rinv;
  const R mr3 = mr * rinv2;
  const R rv = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
  const R mr3t = mr3 * (rv * rinv2);
  if constexpr (FIRST) { // the group's first pair initialises its sums
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
  return r2u;
}

template <int PREC>
__device__ __forceinline__ void load_i(IState<PREC> &st, const ForceArgs &a, int i, bool valid,
                                       int &islot, real_t<PREC> &h2) {
  using R = real_t<PREC>;
  double xi[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0};
  islot = -1;
  h2 = R(-INFINITY);
  if (valid) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xi[d] = a.xi[3 * static_cast<size_t>(i) + d];
      vi[d] = a.vi[3 * static_cast<size_t>(i) + d];
    }
    islot = a.islot[i];
    h2 = static_cast<R>(a.h2[i]);
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

// Per-pair path for tiles holding an own slot or the ragged end: the pair
// terms go through group sums of kGroup pairs (float32 variants) before the
// tile sums, as on the grouped path.
template <int PREC, bool NBL>
struct MaskedRun {
  using R = real_t<PREC>;
  Sums<R> g;
  int n = 0;
  __device__ __forceinline__ void start() {
    g.zero();
    n = 0;
  }
  __device__ __forceinline__ void step(const IState<PREC> &st, Sums<R> &ts, const float4 *rec, int jslot,
                                       int islot, R eps2, R h2, R &best, int &bslot, int *nb_count,
                                       int *nb_row) {
    if constexpr (PREC == G6MI_PREC_FP64) {
      pair<PREC, true, NBL>(st, ts, rec, jslot, islot, eps2, h2, best, bslot, nb_count, nb_row);
    } else {
      pair<PREC, true, NBL>(st, g, rec, jslot, islot, eps2, h2, best, bslot, nb_count, nb_row);
      if (++n == kGroup) {
        ts.add(g);
        start();
      }
    }
  }
  __device__ __forceinline__ void finish(Sums<R> &ts) {
    if constexpr (PREC != G6MI_PREC_FP64) ts.add(g);
  }
};


__device__ __forceinline__ void nb_append(int *__restrict__ nb_count, int *__restrict__ nb_slot,
                                          int i, int jslot) {
  const int pos = atomicAdd(nb_count + i, 1);
  if (pos < kNbMax) nb_slot[static_cast<size_t>(i) * kNbMax + pos] = jslot;
}

// Wide blocks: each lane owns two i-particles (i0 = base + tid and
// i1 = base + 256 + tid, 512 per workgroup) and every lane of a wave reads
// the same j-record from LDS (a broadcast), so one LDS record serves 128
// pairs.  Grid: x = i-blocks of 512, y = j-splits.
//
// The j-loop runs in groups of kGroup records.  Nearest neighbour: one
// min() per pair; once per group the group minimum is compared with the
// running best and the group's first slot remembered; the exact slot is
// recovered at the end by re-examining that one group (first minimum wins,
// as in a sequential scan).  Neighbour lists need no per-pair test: a group
// holds a neighbour of i exactly when its minimum r^2 is below h_i^2, and
// only such groups are re-examined.
// Tiles that contain an i-particle's own slot, and the ragged last tile,
// take the per-pair path with explicit self exclusion.

// Register budget: G6MI_WIDE_WAVES waves per SIMD for the float32
// variants; float64 state takes twice the registers, so one wave fewer.
template <int PREC> constexpr int wide_waves() {
  return G6MI_WIDE_WAVES <= 1 ? 1 : (PREC == G6MI_PREC_FP64 ? G6MI_WIDE_WAVES - 1 : G6MI_WIDE_WAVES);
}

template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG, wide_waves<PREC>()) void force_wide(ForceArgs a) {
  using R = real_t<PREC>;
  constexpr int REC = rec4<PREC>();
  constexpr int kLoads = kTile * REC / kWG; // 16-byte loads per lane per tile
  static_assert(kTile * REC % kWG == 0, "whole loads per lane");
  __shared__ __attribute__((aligned(16))) float4 tile[kTile * REC];

  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * (2 * kWG) + tid;
  const int i1 = i0 + kWG;
  const bool v0 = i0 < a.ni, v1 = i1 < a.ni;
  IState<PREC> s0, s1;
  int slot0, slot1;
  R h20, h21;
  load_i<PREC>(s0, a, i0, v0, slot0, h20);
  load_i<PREC>(s1, a, i1, v1, slot1, h21);
  const R eps2 = static_cast<R>(a.eps2);
  Totals t0 = {{0, 0, 0}, {0, 0, 0}, 0}, t1 = {{0, 0, 0}, {0, 0, 0}, 0};
  Sums<R> ts0, ts1; // tile sums
  ts0.zero();
  ts1.zero();
  // nearest neighbour: fast-path best r^2 and its group; exact path best
  R gbest0 = R(INFINITY), gbest1 = R(INFINITY);
  int grp0 = -1, grp1 = -1;
  R ebest0 = R(INFINITY), ebest1 = R(INFINITY);
  int eslot0 = -1, eslot1 = -1;

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int tb = blockIdx.y * per;
  const int te = min(ntiles, tb + per);
  const float4 *jp = static_cast<const float4 *>(a.jpred);

  for (int tt = tb; tt < te; ++tt) {
    const int jbase = tt * kTile;
    const int cnt = min(kTile, a.nj - jbase);
    __syncthreads();
    {
      // coalesced 16-byte loads of the tile into LDS (records < nj only)
      const float4 *src = jp + static_cast<size_t>(jbase) * REC;
      const int n4 = cnt * REC;
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const int idx = q * kWG + tid;
        if (idx < n4) tile[idx] = src[idx];
      }
    }
    __syncthreads();
    const bool self_here = (slot0 >= jbase && slot0 < jbase + cnt) || (slot1 >= jbase && slot1 < jbase + cnt);
    if (cnt < kTile || __any(self_here)) {
      MaskedRun<PREC, NBL> r0, r1;
      r0.start();
      r1.start();
      for (int jj = 0; jj < cnt; ++jj) {
        r0.step(s0, ts0, tile + jj * REC, jbase + jj, slot0, eps2, h20, ebest0, eslot0,
                a.nb_count + (v0 ? i0 : 0), a.nb_slot + static_cast<size_t>(v0 ? i0 : 0) * kNbMax);
        r1.step(s1, ts1, tile + jj * REC, jbase + jj, slot1, eps2, h21, ebest1, eslot1,
                a.nb_count + (v1 ? i1 : 0), a.nb_slot + static_cast<size_t>(v1 ? i1 : 0) * kNbMax);
      }
      r0.finish(ts0);
      r1.finish(ts1);
    } else {
      // bit k of nbm0 / nbm1: group k holds a neighbour of i0 / i1
      unsigned nbm0 = 0u, nbm1 = 0u;
#pragma unroll G6MI_GROUP_UNROLL
      for (int g = 0; g < kTile; g += kGroup) {
        R m0 = R(INFINITY), m1 = R(INFINITY);
        if constexpr (PREC == G6MI_PREC_FP64) {
#pragma unroll
          for (int u = 0; u < kGroup; ++u) {
            const float4 *rec = tile + (g + u) * REC;
            m0 = fmin(m0, pair_core<PREC>(s0, ts0, rec, eps2));
            m1 = fmin(m1, pair_core<PREC>(s1, ts1, rec, eps2));
          }
        } else {
          Sums<R> g0, g1; // group sums, set by the group's first pair
          m0 = pair_core<PREC, true>(s0, g0, tile + g * REC, eps2);
          m1 = pair_core<PREC, true>(s1, g1, tile + g * REC, eps2);
#pragma unroll
          for (int u = 1; u < kGroup; ++u) {
            const float4 *rec = tile + (g + u) * REC;
            m0 = fmin(m0, pair_core<PREC>(s0, g0, rec, eps2));
            m1 = fmin(m1, pair_core<PREC>(s1, g1, rec, eps2));
          }
          ts0.add(g0);
          ts1.add(g1);
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
          // the group minimum also tells whether any record is a neighbour
          nbm0 |= (m0 < h20 ? 1u : 0u) << (g / kGroup);
          nbm1 |= (m1 < h21 ? 1u : 0u) << (g / kGroup);
        }
      }
      if constexpr (NBL) {
        // rare: append the neighbours of the flagged groups
        while (nbm0 | nbm1) {
          const int k = __builtin_ctz(nbm0 | nbm1);
          const unsigned bit = 1u << k;
          for (int u = 0; u < kGroup; ++u) {
            const int jj = k * kGroup + u;
            const float4 *rec = tile + jj * REC;
            if ((nbm0 & bit) && r2_of<PREC>(s0, rec) < h20) nb_append(a.nb_count, a.nb_slot, i0, jbase + jj);
            if ((nbm1 & bit) && r2_of<PREC>(s1, rec) < h21) nb_append(a.nb_count, a.nb_slot, i1, jbase + jj);
          }
          nbm0 &= ~bit;
          nbm1 &= ~bit;
        }
      }
    }
    fold(ts0, t0);
    fold(ts1, t1);
  }

  // exact slot of the fast-path nearest neighbour: re-examine its group
  // (records are read from global memory; every slot is < nj)
  auto resolve = [&](const IState<PREC> &st, int grp, R &best, int &bslot) {
    if (grp < 0) return;
    for (int u = 0; u < kGroup; ++u) {
      const R r = r2_of<PREC>(st, jp + static_cast<size_t>(grp + u) * REC);
      if (r < best || (r == best && grp + u < bslot)) {
        best = r;
        bslot = grp + u;
      }
    }
  };
  resolve(s0, grp0, ebest0, eslot0);
  resolve(s1, grp1, ebest1, eslot1);

  const size_t ni = static_cast<size_t>(a.ni);
  auto store = [&](int i, const Totals &t, R best, int bslot) {
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = t.acc[d];
      p[(3 + d) * ni] = t.jrk[d];
    }
    p[6 * ni] = t.pot;
    a.nn_r2[blockIdx.y * ni + i] = static_cast<double>(best);
    a.nn_slot[blockIdx.y * ni + i] = bslot;
  };
  if (v0) store(i0, t0, ebest0, eslot0);
  if (v1) store(i1, t1, ebest1, eslot1);
}

// Small blocks: ipw i-particles per workgroup (a power of two, at most 256)
// and L = 256 / ipw lanes per i-particle.  Lane tid handles i-particle
// (tid mod ipw) and records sub, sub + L, sub + 2L, ... of every tile, with
// sub = tid / ipw: when the block is smaller than the workgroup the spare
// lanes split the j-tile among themselves (Sec. 2.3, Fig. accMP1).  For
// ipw >= 64 every lane of a wave reads the same record (an LDS broadcast).
// Full tiles without an own slot use the grouped path of force_wide
// (one min() per pair for the nearest neighbour, one neighbour bit per
// group); the L lane sums of an i-particle are added in a fixed order.
// Grid: x = i-blocks, y = j-splits.
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG) void force_kernel(ForceArgs a) {
  using R = real_t<PREC>;
  constexpr int REC = rec4<PREC>();
  constexpr int kLoads = kTile * REC / kWG;
  constexpr int kRedBytes = kWG * 9 * 8; // 7 sums + r2 + slot per lane
  constexpr int kTileBytes = kTile * REC * 16;
  constexpr int kLdsBytes = kRedBytes > kTileBytes ? kRedBytes : kTileBytes;
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  float4 *tile = reinterpret_cast<float4 *>(lds);

  const int tid = threadIdx.x;
  const int ipw = a.ipw;
  const int log2L = 8 - a.log2ipw;
  const int L = 1 << log2L;
  const int il = tid & (ipw - 1);
  const int sub = tid >> a.log2ipw;
  const int i = blockIdx.x * ipw + il;
  const bool valid = i < a.ni;

  IState<PREC> st;
  int slot;
  R h2;
  load_i<PREC>(st, a, i, valid, slot, h2);
  const R eps2 = static_cast<R>(a.eps2);
  Totals t = {{0, 0, 0}, {0, 0, 0}, 0};
  Sums<R> ts; // tile sums
  ts.zero();
  R gbest = R(INFINITY), ebest = R(INFINITY);
  int grp = -1, eslot = -1;
  int *nb_cnt = a.nb_count + (valid ? i : 0);
  int *nb_row = a.nb_slot + static_cast<size_t>(valid ? i : 0) * kNbMax;
  const int K = kTile >> log2L; // records per lane in a full tile

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int tb = blockIdx.y * per;
  const int te = min(ntiles, tb + per);
  const float4 *jp = static_cast<const float4 *>(a.jpred);

  for (int tt = tb; tt < te; ++tt) {
    const int jbase = tt * kTile;
    const int cnt = min(kTile, a.nj - jbase);
    __syncthreads();
    {
      const float4 *src = jp + static_cast<size_t>(jbase) * REC;
      const int n4 = cnt * REC;
#pragma unroll
      for (int q = 0; q < kLoads; ++q) {
        const int idx = q * kWG + tid;
        if (idx < n4) tile[idx] = src[idx];
      }
    }
    __syncthreads();
    const bool self_here = slot >= jbase && slot < jbase + cnt;
    if (cnt < kTile || K < kGroup || __any(self_here)) {
      MaskedRun<PREC, NBL> run;
      run.start();
      for (int jj = sub; jj < cnt; jj += L)
        run.step(st, ts, tile + jj * REC, jbase + jj, slot, eps2, h2, ebest, eslot, nb_cnt, nb_row);
      run.finish(ts);
    } else {
      unsigned nbm = 0u;
      for (int k0 = 0; k0 < K; k0 += kGroup) {
        R m = R(INFINITY);
        if constexpr (PREC == G6MI_PREC_FP64) {
#pragma unroll
          for (int u = 0; u < kGroup; ++u)
            m = fmin(m, pair_core<PREC>(st, ts, tile + (sub + ((k0 + u) << log2L)) * REC, eps2));
        } else {
          Sums<R> gs; // group sums, set by the group's first pair
          m = pair_core<PREC, true>(st, gs, tile + (sub + (k0 << log2L)) * REC, eps2);
#pragma unroll
          for (int u = 1; u < kGroup; ++u)
            m = fmin(m, pair_core<PREC>(st, gs, tile + (sub + ((k0 + u) << log2L)) * REC, eps2));
          ts.add(gs);
        }
        if (m < gbest) {
          gbest = m;
          grp = jbase + sub + (k0 << log2L);
        }
        if constexpr (NBL) nbm |= (m < h2 ? 1u : 0u) << (k0 / kGroup);
      }
      if constexpr (NBL) {
        while (nbm) { // rare: append the neighbours of the flagged groups
          const int g = __builtin_ctz(nbm);
          nbm &= nbm - 1u;
          for (int u = 0; u < kGroup; ++u) {
            const int jj = sub + ((g * kGroup + u) << log2L);
            if (r2_of<PREC>(st, tile + jj * REC) < h2) nb_append(a.nb_count, a.nb_slot, i, jbase + jj);
          }
        }
      }
    }
    fold(ts, t);
  }

  // exact slot of the grouped-path nearest neighbour: re-examine its group
  if (grp >= 0) {
    for (int u = 0; u < kGroup; ++u) {
      const int js = grp + (u << log2L); // within one full tile, so < nj
      const R r = r2_of<PREC>(st, jp + static_cast<size_t>(js) * REC);
      if (r < ebest || (r == ebest && js < eslot)) {
        ebest = r;
        eslot = js;
      }
    }
  }

  double bestd = static_cast<double>(ebest);
  int bslot = eslot;
  if (L > 1) {
    __syncthreads();
    double *red = reinterpret_cast<double *>(lds); // [9][kWG]
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[d * kWG + tid] = t.acc[d];
      red[(3 + d) * kWG + tid] = t.jrk[d];
    }
    red[6 * kWG + tid] = t.pot;
    red[7 * kWG + tid] = bestd;
    reinterpret_cast<int *>(red + 8 * kWG)[tid] = bslot;
    __syncthreads();
    if (sub == 0) {
      for (int q = 1; q < L; ++q) {
        const int o = q * ipw + il;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          t.acc[d] += red[d * kWG + o];
          t.jrk[d] += red[(3 + d) * kWG + o];
        }
        t.pot += red[6 * kWG + o];
        const double r2o = red[7 * kWG + o];
        const int so = reinterpret_cast<const int *>(red + 8 * kWG)[o];
        if (so >= 0 && (r2o < bestd || (r2o == bestd && (bslot < 0 || so < bslot)))) {
          bestd = r2o;
          bslot = so;
        }
      }
    }
  }
  if (sub == 0 && valid) {
    const size_t ni = static_cast<size_t>(a.ni);
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = t.acc[d];
      p[(3 + d) * ni] = t.jrk[d];
    }
    p[6 * ni] = t.pot;
    a.nn_r2[blockIdx.y * ni + i] = bestd;
    a.nn_slot[blockIdx.y * ni + i] = bslot;
  }
}

// --------------------------------------------------------------- reduction

// One thread per i-particle: float64 sum over the j-splits in split order,
// lexicographic (r2, slot) minimum for the nearest neighbour, and the
// neighbour list turned from slots into particle indices sorted ascending.
// status[kStatusFlags] bit 0: a non-finite output; bit 1: a neighbour list
// overflowed.  Overflowed i-particles are queued in ovf_list for
// nb_exact_kernel (status[kStatusOverflowCount] of them).
__global__ __launch_bounds__(256) void reduce_kernel(
    int nsplit, int ni, const double *__restrict__ part,
    const double *__restrict__ nn_r2, const int *__restrict__ nn_slot,
    const int *__restrict__ jindex, const int *__restrict__ nb_count,
    int *__restrict__ nb_slot, int nbl, double *__restrict__ acc,
    double *__restrict__ jerk, double *__restrict__ pot, int *__restrict__ nnb,
    double *__restrict__ r2nn, int *__restrict__ status, int *__restrict__ ovf_list) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ni) return;
  const size_t n = static_cast<size_t>(ni);
  double s[7] = {0, 0, 0, 0, 0, 0, 0};
  double best = INFINITY;
  int bslot = -1;
  for (int q = 0; q < nsplit; ++q) {
    const double *p = part + static_cast<size_t>(q) * 7 * n + i;
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += p[c * n];
    const double r2 = nn_r2[q * n + i];
    const int sl = nn_slot[q * n + i];
    if (sl >= 0 && (r2 < best || (r2 == best && (bslot < 0 || sl < bslot)))) {
      best = r2;
      bslot = sl;
    }
  }
  bool finite = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    acc[3 * static_cast<size_t>(i) + d] = s[d];
    jerk[3 * static_cast<size_t>(i) + d] = s[3 + d];
    finite = finite && isfinite(s[d]) && isfinite(s[3 + d]);
  }
  pot[i] = -s[6];
  finite = finite && isfinite(s[6]);
  if (nnb) nnb[i] = bslot >= 0 ? jindex[bslot] : -1;
  if (r2nn) r2nn[i] = bslot >= 0 ? best : INFINITY;
  int fl = finite ? 0 : 1;
  if (nbl) {
    const int cnt = nb_count[i];
    int *row = nb_slot + static_cast<size_t>(i) * kNbMax;
    if (cnt > kNbMax) { // kept set decided later by nb_exact_kernel
      fl |= 2;
      ovf_list[atomicAdd(status + kStatusOverflowCount, 1)] = i;
      if (fl) atomicOr(status + kStatusFlags, fl);
      return;
    }
    const int k = cnt;
    for (int a = 0; a < k; ++a) row[a] = jindex[row[a]];
    for (int a = 1; a < k; ++a) { // insertion sort: lists are short
      const int key = row[a];
      int b = a - 1;
      while (b >= 0 && row[b] > key) {
        row[b + 1] = row[b];
        --b;
      }
      row[b + 1] = key;
    }
  }
  if (fl) atomicOr(status + kStatusFlags, fl);
}

// --------------------------------------------- neighbour-list overflow

// For every i-particle whose neighbour count exceeded kNbMax, rebuild its
// list as the kNbMax smallest particle indices among its neighbours, in
// ascending order (the oracle's convention).  One workgroup per queued
// i-particle, grid-strided over the queue.  The neighbour test is the one of
// the interaction kernels (same separation and r^2 arithmetic), repeated
// over all nj slots: a binary search on the index threshold T counts the
// neighbours with index below T (indices biased to unsigned order), then
// the kNbMax of them below the final T are collected and rank-sorted.
template <int PREC>
__global__ __launch_bounds__(kWG) void nb_exact_kernel(ForceArgs a, const int *__restrict__ jindex,
                                                        const int *__restrict__ status,
                                                        const int *__restrict__ ovf_list) {
  using R = real_t<PREC>;
  constexpr int REC = rec4<PREC>();
  __shared__ unsigned s_cnt;
  __shared__ int s_keep[kNbMax];
  const int tid = threadIdx.x;
  const float4 *jp = static_cast<const float4 *>(a.jpred);
  const int novf = status[kStatusOverflowCount];
  for (int q = blockIdx.x; q < novf; q += gridDim.x) {
    const int i = ovf_list[q];
    IState<PREC> st;
    int slot;
    R h2;
    load_i<PREC>(st, a, i, true, slot, h2);
    auto below = [&](unsigned long long T, bool collect) -> unsigned {
      __syncthreads();
      if (tid == 0) s_cnt = 0u;
      __syncthreads();
      unsigned c = 0u;
      for (int js = tid; js < a.nj; js += kWG) {
        const unsigned key = static_cast<unsigned>(jindex[js]) ^ 0x80000000u;
        if (js != slot && key < T && r2_of<PREC>(st, jp + static_cast<size_t>(js) * REC) < h2) {
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
    // smallest T with at least kNbMax neighbours below it
    unsigned long long lo = 0ull, hi = 1ull << 32;
    while (hi - lo > 1ull) {
      const unsigned long long mid = (lo + hi) >> 1;
      if (below(mid, false) >= static_cast<unsigned>(kNbMax)) hi = mid;
      else lo = mid;
    }
    const unsigned got = below(hi, true);
    const int n = got < static_cast<unsigned>(kNbMax) ? static_cast<int>(got) : kNbMax;
    int *row = a.nb_slot + static_cast<size_t>(i) * kNbMax;
    if (tid < n) { // rank sort; equal values ranked by position
      const int v = s_keep[tid];
      int r = 0;
      for (int u = 0; u < n; ++u) r += (s_keep[u] < v) | ((s_keep[u] == v) & (u < tid));
      row[r] = v;
    }
  }
}

// ------------------------------------------------------------ j-memory I/O

__global__ __launch_bounds__(256) void scatter_kernel(int nd, const int *__restrict__ slots,
                                                      const double *__restrict__ rec, JMem jm) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nd) return;
  const size_t k = static_cast<size_t>(slots[q]);
  if (k >= jm.cap) return;
  const double *r = rec + 16 * static_cast<size_t>(q);
  jm.t[k] = r[0];
  jm.m[k] = r[1];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    jm.x[d * jm.cap + k] = r[2 + d];
    jm.v[d * jm.cap + k] = r[5 + d];
    jm.a2[d * jm.cap + k] = r[8 + d];
    jm.j6[d * jm.cap + k] = r[11 + d];
  }
  jm.index[k] = static_cast<int>(r[14]);
}

__global__ __launch_bounds__(256) void load_kernel(int nj, const double *__restrict__ t,
                                                   const double *__restrict__ m,
                                                   const int *__restrict__ index,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ v,
                                                   const double *__restrict__ a2,
                                                   const double *__restrict__ j6, JMem jm) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nj) return;
  jm.t[k] = t[k];
  jm.m[k] = m[k];
  jm.index[k] = index[k];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    jm.x[d * jm.cap + k] = x[3 * static_cast<size_t>(k) + d];
    jm.v[d * jm.cap + k] = v[3 * static_cast<size_t>(k) + d];
    jm.a2[d * jm.cap + k] = a2[3 * static_cast<size_t>(k) + d];
    jm.j6[d * jm.cap + k] = j6[3 * static_cast<size_t>(k) + d];
  }
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks_for(long n) { return static_cast<unsigned>((n + 255) / 256); }

hipError_t launch_predict(int prec, int nj, double ti, const JMem &jm, void *out,
                          int *nb_count, int ni, int *status, hipStream_t s) {
  long n = nj > ni ? nj : ni;
  if (n < kStatusWords) n = kStatusWords;
  if (n <= 0) return hipSuccess;
  const dim3 grid(blocks_for(n)), block(256);
  switch (prec) {
  case G6MI_PREC_FP32:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP32>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni, status);
    break;
  case G6MI_PREC_DS:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_DS>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni, status);
    break;
  default:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP64>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni, status);
  }
  return hipGetLastError();
}

template <int PREC>
static void launch_force_prec(bool nbl, const ForceArgs &a, dim3 grid, hipStream_t s) {
  if (a.ipw == 2 * kWG) {
    if (nbl)
      hipLaunchKernelGGL((force_wide<PREC, true>), grid, dim3(kWG), 0, s, a);
    else
      hipLaunchKernelGGL((force_wide<PREC, false>), grid, dim3(kWG), 0, s, a);
  } else if (nbl)
    hipLaunchKernelGGL((force_kernel<PREC, true>), grid, dim3(kWG), 0, s, a);
  else
    hipLaunchKernelGGL((force_kernel<PREC, false>), grid, dim3(kWG), 0, s, a);
}

hipError_t launch_force(int prec, bool nbl, const ForceArgs &a, int nsplit, hipStream_t s) {
  if (a.ni <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((a.ni + a.ipw - 1) / a.ipw), static_cast<unsigned>(nsplit));
  switch (prec) {
  case G6MI_PREC_FP32: launch_force_prec<G6MI_PREC_FP32>(nbl, a, grid, s); break;
  case G6MI_PREC_DS: launch_force_prec<G6MI_PREC_DS>(nbl, a, grid, s); break;
  default: launch_force_prec<G6MI_PREC_FP64>(nbl, a, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(int nsplit, int ni, const double *part, const double *nn_r2,
                         const int *nn_slot, const int *jindex, int *nb_count, int *nb_slot,
                         bool nbl, double *acc, double *jerk, double *pot, int *nnb,
                         double *r2nn, int *status, int *ovf_list, hipStream_t s) {
  if (ni <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(ni)), dim3(256), 0, s, nsplit, ni, part,
                     nn_r2, nn_slot, jindex, nb_count, nb_slot, nbl ? 1 : 0, acc, jerk, pot,
                     nnb, r2nn, status, ovf_list);
  return hipGetLastError();
}

template <int PREC>
static void launch_exact_prec(const ForceArgs &a, const int *jindex, const int *status,
                              const int *ovf_list, int ngroups, hipStream_t s) {
  hipLaunchKernelGGL(nb_exact_kernel<PREC>, dim3(ngroups), dim3(kWG), 0, s, a, jindex,
                     status, ovf_list);
}

hipError_t launch_nb_exact(int prec, const ForceArgs &a, const int *jindex, const int *status,
                           const int *ovf_list, int novf, hipStream_t s) {
  if (novf <= 0) return hipSuccess;
  const int ngroups = novf < 1024 ? novf : 1024;
  switch (prec) {
  case G6MI_PREC_FP32: launch_exact_prec<G6MI_PREC_FP32>(a, jindex, status, ovf_list, ngroups, s); break;
  case G6MI_PREC_DS: launch_exact_prec<G6MI_PREC_DS>(a, jindex, status, ovf_list, ngroups, s); break;
  default: launch_exact_prec<G6MI_PREC_FP64>(a, jindex, status, ovf_list, ngroups, s);
  }
  return hipGetLastError();
}

hipError_t launch_scatter(int nd, const int *slots, const double *rec, const JMem &jm,
                          hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(nd)), dim3(256), 0, s, nd, slots, rec, jm);
  return hipGetLastError();
}

hipError_t launch_load(int nj, const double *t, const double *m, const int *index,
                       const double *x, const double *v, const double *a2, const double *j6,
                       const JMem &jm, hipStream_t s) {
  if (nj <= 0) return hipSuccess;
  hipLaunchKernelGGL(load_kernel, dim3(blocks_for(nj)), dim3(256), 0, s, nj, t, m, index, x, v,
                     a2, j6, jm);
  return hipGetLastError();
}

} // namespace g6mi
