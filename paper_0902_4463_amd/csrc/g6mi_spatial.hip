// Spatially ordered evaluation of large double-single blocks.
//
// The double-single separation of Eq. (3) costs nine float32 operations per
// pair against three for a plain float32 difference, and it is needed only
// where a float32 difference would lose the digits: between particles close
// compared with their distance from the origin of the coordinates.  Here the
// j-records and the i-block are put in a space-filling (Morton) order, so
// that a tile of 256 consecutive records and a workgroup's 512 i-particles
// each occupy a compact box.  For a tile whose box is farther from the
// i-box than K times the tile's own radius r_t, both sides are re-expressed
// relative to the tile's centre c and the pairs use float32 differences of
// those small coordinates.
//
// Error of the far separation.  A = x_j - c and B = x_i - c are formed once
// per tile (per record and per i-particle, not per pair) in float64 from the
// double-single values, where hi + lo and c_hi + c_lo are exact, and rounded
// once to float32; the pair then takes d = fl(A' - B').  With |A| <= r_t and
// the boxes' gap g >= K r_t (so |D| >= g >= K r_t, D = x_j - x_i),
//   |d - D| <= u (|A| + |B| + |D|) <= u (r_t + (r_t + |D|) + |D|)
//            <= 2 (1 + 1/K) u |D|,   u = 2^-24,
// against 2 u |D| for Eq. (3) (both up to O(u^2) terms, and both relative to
// the double-single positions themselves).  The tile and i-boxes are
// rounded outwards from hi + lo, so that they contain the double-single
// positions and the computed gap never exceeds the true distance by more
// than its own float32 rounding.  Nearer tiles, tiles holding an
// i-particle's own record and ragged tiles take the double-single path.
//
// Far tiles mostly need no neighbour work.  Each particle's nearest-
// neighbour search starts below a bound taken from the record next to its
// own in the sorted order (WideLanes::seed_nn), and a wave whose particles
// all lie farther from a far tile than that bound and the neighbour radius
// allow walks the tile without the group minima and flags (far_quiet,
// tile_far<false>): the same sums, about two thirds of an instruction per
// pair fewer.
//
//   sp_init_kernel, sp_bbox_kernel    bounding box of the predicted j (hi parts)
//   sp_jkeys_kernel, sp_ikeys_kernel  30-bit Morton keys of j and i positions
//   (rocPRIM radix sort of (key, index) pairs)
//   sp_gather_kernel                  records in sorted order, slot in the
//                                     second float4's w; position of each slot
//   sp_tile_kernel                    per tile: centre (double-single),
//                                     radius, box
//   force_spatial<NBL>                the wide interaction kernel over the
//                                     sorted records and i-blocks

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "g6mi_device.h"

namespace g6mi {

// Order-preserving keys of floats for atomic min / max.
__device__ __forceinline__ unsigned fkey(float x) {
  const unsigned b = __float_as_uint(x);
  return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fkey_value(unsigned k) {
  return __uint_as_float((k >> 31) ? (k & 0x7fffffffu) : ~k);
}

__global__ __launch_bounds__(64) void sp_init_kernel(unsigned *__restrict__ box) {
  const int t = threadIdx.x;
  if (t < 3) box[t] = 0xffffffffu; // min keys
  else if (t < 6) box[t] = 0u;     // max keys
}

// Workgroup minimum / maximum of six floats held by every thread, combined
// into box[] with one atomic each (thread 0).
__device__ __forceinline__ void box_reduce(float lo[3], float hi[3], unsigned *__restrict__ box) {
  __shared__ float s[6][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fminf(lo[d], __shfl_xor(lo[d], off));
      hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], off));
    }
  if (lane == 0)
    for (int d = 0; d < 3; ++d) {
      s[d][wave] = lo[d];
      s[3 + d][wave] = hi[d];
    }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    atomicMin(box + d, fkey(fminf(fminf(s[d][0], s[d][1]), fminf(s[d][2], s[d][3]))));
    atomicMax(box + 3 + d, fkey(fmaxf(fmaxf(s[3 + d][0], s[3 + d][1]), fmaxf(s[3 + d][2], s[3 + d][3]))));
  }
}

// Grid-strided over the records: a few hundred workgroups, so that the six
// box words take few atomics (one workgroup per 256 records serialised
// about 25000 of them on six addresses: 0.1 ms at 2^20 records).
__global__ __launch_bounds__(256) void sp_bbox_kernel(int nj, const float4 *__restrict__ rec,
                                                      unsigned *__restrict__ box) {
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = blockIdx.x * 256 + threadIdx.x; k < nj; k += gridDim.x * 256) {
    const float4 p = rec[3 * static_cast<size_t>(k)];
    lo[0] = fminf(lo[0], p.x);
    lo[1] = fminf(lo[1], p.y);
    lo[2] = fminf(lo[2], p.z);
    hi[0] = fmaxf(hi[0], p.x);
    hi[1] = fmaxf(hi[1], p.y);
    hi[2] = fmaxf(hi[2], p.z);
  }
  box_reduce(lo, hi, box);
}

// 10 bits per axis, interleaved (x lowest).
__device__ __forceinline__ unsigned spread10(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ unsigned morton(float x, float y, float z, const unsigned *__restrict__ box) {
  const float p[3] = {x, y, z};
  unsigned key = 0u;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float lo = fkey_value(box[d]), hi = fkey_value(box[3 + d]);
    const float span = hi - lo;
    float q = span > 0.0f ? (p[d] - lo) * (1024.0f / span) : 0.0f;
    q = fminf(fmaxf(q, 0.0f), 1023.0f); // also catches NaN (fmax/fmin drop it)
    key |= spread10(static_cast<unsigned>(q)) << d;
  }
  return key;
}

__global__ __launch_bounds__(256) void sp_jkeys_kernel(int nj, const float4 *__restrict__ rec,
                                                       const unsigned *__restrict__ box,
                                                       unsigned *__restrict__ keys, int *__restrict__ vals) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= nj) return;
  const float4 p = rec[3 * static_cast<size_t>(k)];
  keys[k] = morton(p.x, p.y, p.z, box);
  vals[k] = k;
}

__global__ __launch_bounds__(256) void sp_ikeys_kernel(int ni, const double *__restrict__ xi,
                                                       const unsigned *__restrict__ box,
                                                       unsigned *__restrict__ keys, int *__restrict__ vals) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ni) return;
  const double *x = xi + 3 * static_cast<size_t>(i);
  keys[i] = morton(static_cast<float>(x[0]), static_cast<float>(x[1]), static_cast<float>(x[2]), box);
  vals[i] = i;
}

// Record at sorted position p = record of slot perm[p], the slot stored in
// the w of its second float4; inv[slot] = position.
__global__ __launch_bounds__(256) void sp_gather_kernel(int nj, const int *__restrict__ perm,
                                                        const float4 *__restrict__ src,
                                                        float4 *__restrict__ dst, int *__restrict__ inv) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nj) return;
  const int k = perm[p];
  const size_t s = 3 * static_cast<size_t>(k), d = 3 * static_cast<size_t>(p);
  float4 lo = src[s + 1];
  lo.w = __int_as_float(k);
  dst[d] = src[s];
  dst[d + 1] = lo;
  dst[d + 2] = src[s + 2];
  inv[k] = p;
}

// i-state at sorted position q = that of row iperm[q], and spos[q] = the
// sorted position of its own j-record (-1 without one): the force kernel then
// reads its i-particles contiguously.
__global__ __launch_bounds__(256) void sp_igather_kernel(int ni, int nj, const int *__restrict__ iperm,
                                                         const int *__restrict__ inv,
                                                         const double *__restrict__ xi,
                                                         const double *__restrict__ vi,
                                                         const double *__restrict__ h2,
                                                         const int *__restrict__ islot, double *__restrict__ sxi,
                                                         double *__restrict__ svi, double *__restrict__ sh2,
                                                         int *__restrict__ sislot, int *__restrict__ spos) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= ni) return;
  const size_t r = static_cast<size_t>(iperm[q]), d = static_cast<size_t>(q);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sxi[3 * d + k] = xi[3 * r + k];
    svi[3 * d + k] = vi[3 * r + k];
  }
  sh2[d] = h2[r];
  const int slot = islot[r];
  sislot[d] = slot;
  spos[d] = (slot >= 0 && slot < nj) ? inv[slot] : -1;
}

// Outward float32 bounds of a double-single value hi + lo (exact in float64):
// down <= hi + lo <= up.
__device__ __forceinline__ void ds_bounds(float hi, float lo, float &down, float &up) {
  const double v = static_cast<double>(hi) + static_cast<double>(lo);
  const float f = static_cast<float>(v);
  down = static_cast<double>(f) > v ? nextafterf(f, -INFINITY) : f;
  up = static_cast<double>(f) < v ? nextafterf(f, INFINITY) : f;
}

// One workgroup per tile of sorted records: the box of the double-single
// positions (rounded outwards), its centre c (float64 midpoint, split
// double-single) and the radius r_t >= max |x - c| over the tile, with x - c
// formed in float64 from hi + lo and c_hi + c_lo (exact sums), rounded up.
// tinfo[4 t .. 4 t + 3] = {c_hi, r_t}, {c_lo, 0}, {box min, 0}, {box max, 0}.
__global__ __launch_bounds__(256) void sp_tile_kernel(int nj, const float4 *__restrict__ rec,
                                                      float4 *__restrict__ tinfo) {
  __shared__ unsigned s_box[6];
  __shared__ float s_c[6];
  __shared__ double s_r[4];
  const int tid = threadIdx.x;
  const int k = blockIdx.x * kTile + tid;
  const bool ok = k < nj;
  if (tid < 6) s_box[tid] = tid < 3 ? 0xffffffffu : 0u;
  __syncthreads();
  float4 ph = make_float4(0, 0, 0, 0), pl = ph;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (ok) {
    ph = rec[3 * static_cast<size_t>(k)];
    pl = rec[3 * static_cast<size_t>(k) + 1];
    ds_bounds(ph.x, pl.x, lo[0], hi[0]);
    ds_bounds(ph.y, pl.y, lo[1], hi[1]);
    ds_bounds(ph.z, pl.z, lo[2], hi[2]);
  }
  box_reduce(lo, hi, s_box);
  __syncthreads();
  if (tid < 3) {
    const double c = 0.5 * (static_cast<double>(fkey_value(s_box[tid])) + static_cast<double>(fkey_value(s_box[3 + tid])));
    const float chi = static_cast<float>(c);
    s_c[tid] = chi;
    s_c[3 + tid] = static_cast<float>(c - static_cast<double>(chi));
  }
  __syncthreads();
  double r = 0.0;
  if (ok) {
    const float h[3] = {ph.x, ph.y, ph.z}, l[3] = {pl.x, pl.y, pl.z};
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a = (static_cast<double>(h[d]) + static_cast<double>(l[d])) -
                       (static_cast<double>(s_c[d]) + static_cast<double>(s_c[3 + d]));
      r2 += a * a;
    }
    r = sqrt(r2);
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off));
  if (lane == 0) s_r[wave] = r;
  __syncthreads();
  if (tid == 0) {
    const double rmax = fmax(fmax(s_r[0], s_r[1]), fmax(s_r[2], s_r[3]));
    // rounded up, with a margin for the float64 rounding of the radius
    const float rt = static_cast<float>(rmax) * (1.0f + 0x1p-20f);
    float4 *o = tinfo + 4 * static_cast<size_t>(blockIdx.x);
    o[0] = make_float4(s_c[0], s_c[1], s_c[2], rt);
    o[1] = make_float4(s_c[3], s_c[4], s_c[5], 0.0f);
    o[2] = make_float4(fkey_value(s_box[0]), fkey_value(s_box[1]), fkey_value(s_box[2]), 0.0f);
    o[3] = make_float4(fkey_value(s_box[3]), fkey_value(s_box[4]), fkey_value(s_box[5]), 0.0f);
  }
}

// The wide DS kernel over sorted records (a.jpred) and the sorted i-state
// (a.xi, a.vi, a.h2, a.islot): workgroup b takes sorted positions 512 b + tid
// and 512 b + 256 + tid; partials go to those positions, neighbour lists to
// the i-particles' own rows iperm[q].
template <bool NBL>
__global__ __launch_bounds__(kWG, wide_waves<G6MI_PREC_DS>()) void force_spatial(ForceArgs a, SpatialArgs sp) {
  constexpr int REC = rec4<G6MI_PREC_DS>();
  constexpr int FREC = rec4<G6MI_PREC_FP32>();
  constexpr int kLoads = kTile * REC / kWG;
  __shared__ __attribute__((aligned(16))) float4 tile[kTile * REC];
  __shared__ __attribute__((aligned(16))) float4 ftile[kTile * FREC];
  __shared__ float s_ib[6];
  const int tid = threadIdx.x;
  const int q0 = blockIdx.x * (2 * kWG) + tid, q1 = q0 + kWG;
  const bool v0 = q0 < a.ni, v1 = q1 < a.ni;
  WideLanes<G6MI_PREC_DS, NBL, true, kSpatialGroup> w;
  w.init(a, v0 ? q0 : 0, v1 ? q1 : 0, v0, v1);
  w.row0 = v0 ? sp.iperm[q0] : 0;
  w.row1 = v1 ? sp.iperm[q1] : 0;
  w.pos0 = v0 ? sp.spos[q0] : -1;
  w.pos1 = v1 ? sp.spos[q1] : -1;
  const float eps2 = static_cast<float>(a.eps2);
  w.seed_nn(static_cast<const float4 *>(a.jpred), a.nj, eps2);

  // box of this workgroup's i-particles (double-single positions, rounded
  // outwards)
  {
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float dn, up;
      if (v0) {
        ds_bounds(w.s0.xh[d], w.s0.xl[d], dn, up);
        lo[d] = fminf(lo[d], dn);
        hi[d] = fmaxf(hi[d], up);
      }
      if (v1) {
        ds_bounds(w.s1.xh[d], w.s1.xl[d], dn, up);
        lo[d] = fminf(lo[d], dn);
        hi[d] = fmaxf(hi[d], up);
      }
    }
    __shared__ unsigned s_ibk[6];
    if (tid < 6) s_ibk[tid] = tid < 3 ? 0xffffffffu : 0u;
    __syncthreads();
    box_reduce(lo, hi, s_ibk);
    __syncthreads();
    if (tid < 6) s_ib[tid] = fkey_value(s_ibk[tid]);
    __syncthreads();
  }

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
    const float4 c_hi = sp.tinfo[4 * static_cast<size_t>(tt)];
    const float4 c_lo = sp.tinfo[4 * static_cast<size_t>(tt) + 1];
    const float4 bmin = sp.tinfo[4 * static_cast<size_t>(tt) + 2];
    const float4 bmax = sp.tinfo[4 * static_cast<size_t>(tt) + 3];
    const bool self_here = (w.pos0 >= jbase && w.pos0 < jbase + cnt) || (w.pos1 >= jbase && w.pos1 < jbase + cnt);
    const int any_self = __syncthreads_or(self_here); // also the barrier after the tile load
    float g2 = 0.0f;
    {
      // the i-box is read from LDS per tile rather than held in registers
      // through the tile loop, where registers are scarce
      const float tl[3] = {bmin.x, bmin.y, bmin.z}, th[3] = {bmax.x, bmax.y, bmax.z};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float gd = fmaxf(0.0f, fmaxf(tl[d] - s_ib[3 + d], s_ib[d] - th[d]));
        g2 += gd * gd;
      }
    }
    const float reach = G6MI_FAR_K * c_hi.w;
    const bool far = cnt == kTile && !any_self && g2 >= reach * reach;
    if (far) {
      // x - c in float64 from the exact sums hi + lo and c_hi + c_lo, rounded
      // once to float32 (the error bound in the header)
      const double c64[3] = {static_cast<double>(c_hi.x) + static_cast<double>(c_lo.x),
                             static_cast<double>(c_hi.y) + static_cast<double>(c_lo.y),
                             static_cast<double>(c_hi.z) + static_cast<double>(c_lo.z)};
      auto rel = [&](float h, float l, int d) {
        return static_cast<float>((static_cast<double>(h) + static_cast<double>(l)) - c64[d]);
      };
      {
        const float4 p = tile[tid * REC], q = tile[tid * REC + 1], v = tile[tid * REC + 2];
        ftile[tid * FREC] = make_float4(rel(p.x, q.x, 0), rel(p.y, q.y, 1), rel(p.z, q.z, 2), p.w);
        ftile[tid * FREC + 1] = make_float4(v.x, v.y, v.z, q.w);
      }
      IState<G6MI_PREC_FP32> f0, f1;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        f0.x[d] = rel(w.s0.xh[d], w.s0.xl[d], d);
        f1.x[d] = rel(w.s1.xh[d], w.s1.xl[d], d);
        f0.v[d] = w.s0.v[d];
        f1.v[d] = w.s1.v[d];
      }
      __syncthreads();
      // a wave whose lanes' neighbour searches the tile cannot touch skips them
      if (__all(w.far_quiet(f0, f1, c_hi.w, eps2)))
        w.template tile_far<false>(ftile, jbase, eps2, f0, f1, a.nb_count, a.nb_slot);
      else
        w.template tile_far<true>(ftile, jbase, eps2, f0, f1, a.nb_count, a.nb_slot);
    } else {
      w.template tile<true>(tile, jbase, cnt, eps2, a.nb_count, a.nb_slot);
    }
  }
  w.resolve(jp, 0); // exact slots from the sorted records in global memory

  const size_t ni = static_cast<size_t>(a.ni);
  auto store = [&](int i, const Totals &t, float best, int bslot) {
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
  if (w.v0) store(q0, w.t0, w.ebest0, w.eslot0);
  if (w.v1) store(q1, w.t1, w.ebest1, w.eslot1);
}

// ---------------------------------------------------------------- launchers

static inline unsigned blocks256(long n) { return static_cast<unsigned>((n + 255) / 256); }

hipError_t spatial_sort_bytes(int n, size_t *bytes) {
  *bytes = 0;
  return rocprim::radix_sort_pairs(nullptr, *bytes, static_cast<const unsigned *>(nullptr),
                                   static_cast<unsigned *>(nullptr), static_cast<const int *>(nullptr),
                                   static_cast<int *>(nullptr), static_cast<size_t>(n), 0, 30);
}

hipError_t launch_spatial_prep(const SpatialBufs &b, int nj, int ni, const void *jpred, const double *xi,
                               const double *vi, const double *h2, const int *islot, hipStream_t s) {
  const float4 *rec = static_cast<const float4 *>(jpred);
  hipLaunchKernelGGL(sp_init_kernel, dim3(1), dim3(64), 0, s, b.box);
  hipLaunchKernelGGL(sp_bbox_kernel, dim3(std::min(blocks256(nj), 512u)), dim3(256), 0, s, nj, rec, b.box);
  hipLaunchKernelGGL(sp_jkeys_kernel, dim3(blocks256(nj)), dim3(256), 0, s, nj, rec, b.box, b.keys_in, b.vals_in);
  size_t bytes = b.temp_bytes;
  hipError_t e = rocprim::radix_sort_pairs(b.temp, bytes, b.keys_in, b.keys_out, b.vals_in, b.jperm,
                                           static_cast<size_t>(nj), 0, 30, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sp_gather_kernel, dim3(blocks256(nj)), dim3(256), 0, s, nj, b.jperm, rec, b.sorted, b.inv);
  hipLaunchKernelGGL(sp_tile_kernel, dim3(static_cast<unsigned>((nj + kTile - 1) / kTile)), dim3(256), 0, s, nj,
                     b.sorted, b.tinfo);
  hipLaunchKernelGGL(sp_ikeys_kernel, dim3(blocks256(ni)), dim3(256), 0, s, ni, xi, b.box, b.keys_in, b.vals_in);
  bytes = b.temp_bytes;
  e = rocprim::radix_sort_pairs(b.temp, bytes, b.keys_in, b.keys_out, b.vals_in, b.iperm, static_cast<size_t>(ni),
                                0, 30, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sp_igather_kernel, dim3(blocks256(ni)), dim3(256), 0, s, ni, nj, b.iperm, b.inv, xi, vi, h2,
                     islot, b.sxi, b.svi, b.sh2, b.sislot, b.spos);
  return hipGetLastError();
}

hipError_t launch_force_spatial(bool nbl, const ForceArgs &a, const SpatialBufs &b, int nsplit, hipStream_t s) {
  if (a.ni <= 0) return hipSuccess;
  ForceArgs as = a; // sorted records and i-state
  as.jpred = b.sorted;
  as.xi = b.sxi;
  as.vi = b.svi;
  as.h2 = b.sh2;
  as.islot = b.sislot;
  SpatialArgs sp;
  sp.iperm = b.iperm;
  sp.spos = b.spos;
  sp.tinfo = b.tinfo;
  const dim3 grid(static_cast<unsigned>((a.ni + 2 * kWG - 1) / (2 * kWG)), static_cast<unsigned>(nsplit));
  if (nbl)
    hipLaunchKernelGGL(force_spatial<true>, grid, dim3(kWG), 0, s, as, sp);
  else
    hipLaunchKernelGGL(force_spatial<false>, grid, dim3(kWG), 0, s, as, sp);
  return hipGetLastError();
}

} // namespace g6mi
