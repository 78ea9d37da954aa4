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
    int *__restrict__ nb_count, int ni) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < ni) nb_count[k] = 0; // fresh neighbour counters for this call
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

// Per-lane state of one i-particle.  FP32/DS sum each tile in float32
// (t*), then add the tile sums into float64 totals (d*); FP64 sums in
// float64 directly.
template <int PREC> struct IState;

template <> struct IState<G6MI_PREC_DS> {
  float xh[3], xl[3], v[3];
  float ta[3], tj1[3], tj2[3], tp;
};
template <> struct IState<G6MI_PREC_FP32> {
  float x[3], v[3];
  float ta[3], tj1[3], tj2[3], tp;
};
template <> struct IState<G6MI_PREC_FP64> {
  double x[3], v[3];
  double ta[3], tj1[3], tj2[3], tp;
};

template <int PREC> using real_t = std::conditional_t<PREC == G6MI_PREC_FP64, double, float>;

// One pair (i, j).  MASK: compare the j-slot with the i-particle's own slot
// and drop the self pair.  NBL: build neighbour lists.
template <int PREC, bool MASK, bool NBL>
__device__ __forceinline__ void pair(IState<PREC> &st, const float4 *__restrict__ rec,
                                     int jslot, int islot, real_t<PREC> eps2,
                                     real_t<PREC> h2, real_t<PREC> &best, int &bslot,
                                     int *__restrict__ nb_count, int *__restrict__ nb_row) {
  using R = real_t<PREC>;
  R dx, dy, dz, dvx, dvy, dvz, mj;
  if constexpr (PREC == G6MI_PREC_DS) {
    const float4 p = rec[0], q = rec[1], w = rec[2];
    // Eq. (3): separation of two DS numbers, 3 float32 operations
    dx = (p.x - st.xh[0]) + (q.x - st.xl[0]);
    dy = (p.y - st.xh[1]) + (q.y - st.xl[1]);
    dz = (p.z - st.xh[2]) + (q.z - st.xl[2]);
    dvx = w.x - st.v[0];
    dvy = w.y - st.v[1];
    dvz = w.z - st.v[2];
    mj = p.w;
  } else if constexpr (PREC == G6MI_PREC_FP32) {
    const float4 p = rec[0], w = rec[1];
    dx = p.x - st.x[0];
    dy = p.y - st.x[1];
    dz = p.z - st.x[2];
    dvx = w.x - st.v[0];
    dvy = w.y - st.v[1];
    dvz = w.z - st.v[2];
    mj = p.w;
  } else {
    const double2 *r2 = reinterpret_cast<const double2 *>(rec);
    const double2 p0 = r2[0], p1 = r2[1], w0 = r2[2], w1 = r2[3];
    dx = p0.x - st.x[0];
    dy = p0.y - st.x[1];
    dz = p1.x - st.x[2];
    dvx = w0.x - st.v[0];
    dvy = w0.y - st.v[1];
    dvz = w1.x - st.v[2];
    mj = p1.y;
  }
  R r2u = dx * dx + dy * dy + dz * dz;
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
  st.tp += mr;
  st.ta[0] += mr3 * dx;
  st.ta[1] += mr3 * dy;
  st.ta[2] += mr3 * dz;
  st.tj1[0] += mr3 * dvx;
  st.tj1[1] += mr3 * dvy;
  st.tj1[2] += mr3 * dvz;
  st.tj2[0] += mr3t * dx;
  st.tj2[1] += mr3t * dy;
  st.tj2[2] += mr3t * dz;
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

// Grid: x = i-blocks of ipw i-particles, y = j-splits.  Lane tid handles
// i-particle (tid mod ipw) of the block and j-records sub, sub + L, ...
// of every tile, with sub = tid / ipw and L = 256 / ipw lanes per
// i-particle.  With ipw >= 64 all lanes of a wave read the same j-record
// (an LDS broadcast).  The L lanes of one i-particle are summed in a fixed
// order at the end.
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG) void force_kernel(ForceArgs a) {
  using R = real_t<PREC>;
  constexpr int REC = rec4<PREC>();
  constexpr int kTileF4 = kTile * REC;
  constexpr int kRedBytes = kWG * 9 * 8; // 7 sums + r2 + slot per lane
  constexpr int kTileBytes = kTileF4 * 16;
  constexpr int kLdsBytes = kRedBytes > kTileBytes ? kRedBytes : kTileBytes;
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  float4 *tile = reinterpret_cast<float4 *>(lds);

  const int tid = threadIdx.x;
  const int ipw = a.ipw;
  const int L = kWG >> a.log2ipw;
  const int il = tid & (ipw - 1);
  const int sub = tid >> a.log2ipw;
  const int i = blockIdx.x * ipw + il;
  const bool ivalid = i < a.ni;

  IState<PREC> st;
  int islot = -1;
  R h2 = R(-INFINITY);
  {
    double xi[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0};
    if (ivalid) {
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
      st.ta[d] = st.tj1[d] = st.tj2[d] = R(0);
    }
    st.tp = R(0);
  }
  const R eps2 = static_cast<R>(a.eps2);
  double acc[3] = {0.0, 0.0, 0.0}, jrk[3] = {0.0, 0.0, 0.0}, pot = 0.0;
  R best = R(INFINITY);
  int bslot = -1;
  int *nb_cnt = a.nb_count + (ivalid ? i : 0);
  int *nb_row = a.nb_slot + static_cast<size_t>(ivalid ? i : 0) * kNbMax;

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int t0 = blockIdx.y * per;
  const int t1 = min(ntiles, t0 + per);
  const float4 *jp = static_cast<const float4 *>(a.jpred);

  for (int tt = t0; tt < t1; ++tt) {
    const int jbase = tt * kTile;
    const int cnt = min(kTile, a.nj - jbase);
    __syncthreads();
    {
      const float4 *src = jp + static_cast<size_t>(jbase) * REC;
      const int n4 = cnt * REC;
      for (int q = tid; q < n4; q += kWG) tile[q] = src[q];
    }
    __syncthreads();
    const bool self_here = islot >= jbase && islot < jbase + cnt;
    if (__any(self_here)) {
      for (int jj = sub; jj < cnt; jj += L)
        pair<PREC, true, NBL>(st, tile + jj * REC, jbase + jj, islot, eps2, h2,
                              best, bslot, nb_cnt, nb_row);
    } else if (cnt == kTile && L == 1) {
#pragma unroll 4
      for (int jj = 0; jj < kTile; ++jj)
        pair<PREC, false, NBL>(st, tile + jj * REC, jbase + jj, islot, eps2,
                               h2, best, bslot, nb_cnt, nb_row);
    } else {
      for (int jj = sub; jj < cnt; jj += L)
        pair<PREC, false, NBL>(st, tile + jj * REC, jbase + jj, islot, eps2,
                               h2, best, bslot, nb_cnt, nb_row);
    }
    // fold the tile sums into the float64 totals
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      acc[d] += static_cast<double>(st.ta[d]);
      jrk[d] += static_cast<double>(st.tj1[d]) - 3.0 * static_cast<double>(st.tj2[d]);
      st.ta[d] = st.tj1[d] = st.tj2[d] = R(0);
    }
    pot += static_cast<double>(st.tp);
    st.tp = R(0);
  }

  double bestd = static_cast<double>(best);
  if (L > 1) {
    __syncthreads();
    double *red = reinterpret_cast<double *>(lds); // [9][kWG]
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red[d * kWG + tid] = acc[d];
      red[(3 + d) * kWG + tid] = jrk[d];
    }
    red[6 * kWG + tid] = pot;
    red[7 * kWG + tid] = bestd;
    reinterpret_cast<int *>(red + 8 * kWG)[tid] = bslot;
    __syncthreads();
    if (sub == 0) {
      for (int q = 1; q < L; ++q) {
        const int o = q * ipw + il;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          acc[d] += red[d * kWG + o];
          jrk[d] += red[(3 + d) * kWG + o];
        }
        pot += red[6 * kWG + o];
        const double r2o = red[7 * kWG + o];
        const int so = reinterpret_cast<const int *>(red + 8 * kWG)[o];
        if (r2o < bestd || (r2o == bestd && so >= 0 && (bslot < 0 || so < bslot))) {
          bestd = r2o;
          bslot = so;
        }
      }
    }
  }
  if (sub == 0 && ivalid) {
    const size_t ni = static_cast<size_t>(a.ni);
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = acc[d];
      p[(3 + d) * ni] = jrk[d];
    }
    p[6 * ni] = pot;
    a.nn_r2[blockIdx.y * ni + i] = bestd;
    a.nn_slot[blockIdx.y * ni + i] = bslot;
  }
}

// ------------------------------------------------- interaction, wide blocks

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

template <int PREC>
__device__ __forceinline__ real_t<PREC> r2_of(const IState<PREC> &st, const float4 *__restrict__ rec) {
  real_t<PREC> d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// The pair terms of Sec. 2.3 added to the tile sums; returns r^2 (without
// softening) for the neighbour search.  No self test: the caller only uses
// it on tiles that hold neither i-particle's own slot.
template <int PREC>
__device__ __forceinline__ real_t<PREC> pair_core(IState<PREC> &st, const float4 *__restrict__ rec,
                                                  real_t<PREC> eps2) {
  using R = real_t<PREC>;
  R d[3], w[3], mj;
  separation<PREC>(st, rec, d, w, mj);
  const R r2u = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const R s = r2u + eps2;
  R rinv;
  if constexpr (PREC == G6MI_PREC_FP64) rinv = rsqrt_f64(s);
  else rinv = __builtin_amdgcn_rsqf(s);
  const R rinv2 = rinv * rinv;
  const R mr = mj * rinv;
  const R mr3 = mr * rinv2;
  const R rv = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
  const R mr3t = mr3 * (rv * rinv2);
  st.tp += mr;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    st.ta[k] += mr3 * d[k];
    st.tj1[k] += mr3 * w[k];
    st.tj2[k] += mr3t * d[k];
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
    st.ta[d] = st.tj1[d] = st.tj2[d] = R(0);
  }
  st.tp = R(0);
}

// Float64 running totals of one i-particle: the tile sums are folded in
// after every tile (float32 variants sum at most kTile terms in float32).
struct Totals {
  double acc[3], jrk[3], pot;
};

template <int PREC>
__device__ __forceinline__ void fold(IState<PREC> &st, Totals &t) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    t.acc[d] += static_cast<double>(st.ta[d]);
    t.jrk[d] += static_cast<double>(st.tj1[d]) - 3.0 * static_cast<double>(st.tj2[d]);
    st.ta[d] = st.tj1[d] = st.tj2[d] = real_t<PREC>(0);
  }
  t.pot += static_cast<double>(st.tp);
  st.tp = real_t<PREC>(0);
}

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
constexpr int kGroup = G6MI_GROUP;
static_assert(kTile / kGroup <= 32, "one mask bit per group");
static_assert(kTile % kGroup == 0, "whole groups per tile");

#if G6MI_WIDE_WAVES > 0
#define G6MI_WIDE_BOUNDS __launch_bounds__(kWG, G6MI_WIDE_WAVES)
#else
#define G6MI_WIDE_BOUNDS __launch_bounds__(kWG)
#endif

template <int PREC, bool NBL>
__global__ G6MI_WIDE_BOUNDS void force_wide(ForceArgs a) {
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
      for (int jj = 0; jj < cnt; ++jj) {
        pair<PREC, true, NBL>(s0, tile + jj * REC, jbase + jj, slot0, eps2, h20, ebest0, eslot0,
                              a.nb_count + (v0 ? i0 : 0),
                              a.nb_slot + static_cast<size_t>(v0 ? i0 : 0) * kNbMax);
        pair<PREC, true, NBL>(s1, tile + jj * REC, jbase + jj, slot1, eps2, h21, ebest1, eslot1,
                              a.nb_count + (v1 ? i1 : 0),
                              a.nb_slot + static_cast<size_t>(v1 ? i1 : 0) * kNbMax);
      }
    } else {
      // bit k of nbm0 / nbm1: group k holds a neighbour of i0 / i1
      unsigned nbm0 = 0u, nbm1 = 0u;
#pragma unroll G6MI_GROUP_UNROLL
      for (int g = 0; g < kTile; g += kGroup) {
        R m0 = R(INFINITY), m1 = R(INFINITY);
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
          const float4 *rec = tile + (g + u) * REC;
          m0 = fmin(m0, pair_core<PREC>(s0, rec, eps2));
          m1 = fmin(m1, pair_core<PREC>(s1, rec, eps2));
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
    fold<PREC>(s0, t0);
    fold<PREC>(s1, t1);
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

// --------------------------------------------------------------- reduction

// One thread per i-particle: float64 sum over the j-splits in split order,
// lexicographic (r2, slot) minimum for the nearest neighbour, and the
// neighbour list turned from slots into particle indices sorted ascending.
// flags bit 0: a non-finite output; bit 1: a neighbour list overflowed.
__global__ __launch_bounds__(256) void reduce_kernel(
    int nsplit, int ni, const double *__restrict__ part,
    const double *__restrict__ nn_r2, const int *__restrict__ nn_slot,
    const int *__restrict__ jindex, const int *__restrict__ nb_count,
    int *__restrict__ nb_slot, int nbl, double *__restrict__ acc,
    double *__restrict__ jerk, double *__restrict__ pot, int *__restrict__ nnb,
    double *__restrict__ r2nn, int *__restrict__ flags) {
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
    const int k = cnt < kNbMax ? cnt : kNbMax;
    if (cnt > kNbMax) fl |= 2;
    int *row = nb_slot + static_cast<size_t>(i) * kNbMax;
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
  if (fl) atomicOr(flags, fl);
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
                          int *nb_count, int ni, hipStream_t s) {
  const long n = nj > ni ? nj : ni;
  if (n <= 0) return hipSuccess;
  const dim3 grid(blocks_for(n)), block(256);
  switch (prec) {
  case G6MI_PREC_FP32:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP32>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni);
    break;
  case G6MI_PREC_DS:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_DS>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni);
    break;
  default:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP64>, grid, block, 0, s, nj, ti, jm.t, jm.m,
                       jm.x, jm.v, jm.a2, jm.j6, jm.cap, out, nb_count, ni);
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
                         double *r2nn, int *flags, hipStream_t s) {
  if (ni <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(ni)), dim3(256), 0, s, nsplit, ni, part,
                     nn_r2, nn_slot, jindex, nb_count, nb_slot, nbl ? 1 : 0, acc, jerk, pot,
                     nnb, r2nn, flags);
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
