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

#include "g6mi_device.h"

#include <mutex>

namespace g6mi {

size_t pred_record_bytes(int prec) {
  switch (prec) {
  case G6MI_PREC_FP32: return 32;
  case G6MI_PREC_DS: return 48;
  default: return 64;
  }
}

// ---------------------------------------------------------------- predictor

// One thread per j-slot: the record of slot k predicted to ti (Sec. 2.2,
// Eq. (1)-(2)) in the layout of the precision variant.  The same launch
// clears the neighbour counters and status words of the calculation.
template <int PREC>
__global__ __launch_bounds__(256) void predict_kernel(int nj, double ti, JMem jm,
                                                      void *__restrict__ out,
                                                      int *__restrict__ nb_count, int ni,
                                                      int *__restrict__ status) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < ni) nb_count[k] = 0; // fresh neighbour counters for this call
  if (k < kStatusWords) status[k] = 0;
  if (k >= nj) return;
  predict_record<PREC>(jm, static_cast<size_t>(k), ti,
                       static_cast<float4 *>(out) + rec4<PREC>() * static_cast<size_t>(k));
}

// ------------------------------------------------- interaction, wide blocks

// Wide blocks (WideLanes): lane tid owns i-particles base + tid and
// base + 256 + tid, 512 per workgroup.  Grid: x = i-blocks of 512,
// y = j-splits; the partials of split y go to part[y][7][ni].
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG, wide_waves<PREC>()) void force_wide(ForceArgs a) {
  constexpr int REC = rec4<PREC>();
  constexpr int kLoads = kTile * REC / kWG; // 16-byte loads per lane per tile
  static_assert(kTile * REC % kWG == 0, "whole loads per lane");
  __shared__ __attribute__((aligned(16))) float4 tile[kTile * REC];

  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * (2 * kWG) + tid;
  const int i1 = i0 + kWG;
  WideLanes<PREC, NBL> w;
  w.init(a, i0, i1, i0 < a.ni, i1 < a.ni);
  const real_t<PREC> eps2 = static_cast<real_t<PREC>>(a.eps2);

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
    // DS: every group goes straight to the float64 totals (see WideLanes::tile)
    w.template tile<PREC == G6MI_PREC_DS, true>(tile, jbase, cnt, eps2, a.nb_count, a.nb_slot);
  }
  // exact slot of the fast-path nearest neighbours: their groups are
  // re-read from global memory (every slot is < nj)
  w.resolve(jp, 0);

  const size_t ni = static_cast<size_t>(a.ni);
  auto store = [&](int i, const Totals &t, real_t<PREC> best, int bslot) {
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
  if (w.v0) store(i0, w.t0, w.ebest0, w.eslot0);
  if (w.v1) store(i1, w.t1, w.ebest1, w.eslot1);
}

// K float4 per lane of a tile of n4 float4 (lane tid holds elements tid,
// tid + 256, ...), in named registers of a plain vector type (an aggregate
// float4 copy would go through the stack).  Loads are clamped to the last
// element so that every lane loads unconditionally; the store writes only
// the elements below n4.
template <int K> struct TileRegs {
  static_assert(K >= 1 && K <= 4, "one to four float4 per lane");
  typedef float v4 __attribute__((ext_vector_type(4)));
  v4 v0, v1, v2, v3;
  __device__ __forceinline__ void load(const float4 *__restrict__ src4, int tid, int n4) {
    const v4 *src = reinterpret_cast<const v4 *>(src4);
    v0 = src[min(tid, n4 - 1)];
    if constexpr (K > 1) v1 = src[min(kWG + tid, n4 - 1)];
    if constexpr (K > 2) v2 = src[min(2 * kWG + tid, n4 - 1)];
    if constexpr (K > 3) v3 = src[min(3 * kWG + tid, n4 - 1)];
  }
  __device__ __forceinline__ void store(float4 *__restrict__ dst4, int tid, int n4) const {
    v4 *dst = reinterpret_cast<v4 *>(dst4);
    if (tid < n4) dst[tid] = v0;
    if constexpr (K > 1)
      if (kWG + tid < n4) dst[kWG + tid] = v1;
    if constexpr (K > 2)
      if (2 * kWG + tid < n4) dst[2 * kWG + tid] = v2;
    if constexpr (K > 3)
      if (3 * kWG + tid < n4) dst[3 * kWG + tid] = v3;
  }
};

// Small blocks (NarrowLane): ipw i-particles per workgroup (a power of two,
// at most 256) and L = 256 / ipw lanes per i-particle; lane tid handles
// i-particle (tid mod ipw) and the records sub, sub + L, ... of every tile,
// sub = tid / ipw.  For ipw >= 64 every lane of a wave reads the same record
// (an LDS broadcast).  The L lane totals of an i-particle are added in a
// fixed order.  Grid: x = i-blocks, y = j-splits.
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG) void force_kernel(ForceArgs a) {
  constexpr int REC = rec4<PREC>();
  constexpr int kLoads = kTile * REC / kWG;
  __shared__ __attribute__((aligned(16))) unsigned char lds[narrow_lds_bytes<PREC>()];
  float4 *tile = reinterpret_cast<float4 *>(lds);

  const int tid = threadIdx.x;
  const int ipw = a.ipw;
  const int il = tid & (ipw - 1);
  const int i = blockIdx.x * ipw + il;
  NarrowLane<PREC, NBL> n;
  n.init(a, i, i < a.ni, tid >> a.log2ipw, 8 - a.log2ipw);
  const real_t<PREC> eps2 = static_cast<real_t<PREC>>(a.eps2);

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int tb = blockIdx.y * per;
  const int te = min(ntiles, tb + per);
  const float4 *jp = static_cast<const float4 *>(a.jpred);

  // The next tile's records are loaded into registers while the current
  // one is evaluated: a block of few i-particles spends little time per
  // tile, too little to cover the load on its own.
  TileRegs<kLoads> nxt;
  if (tb < te) nxt.load(jp + static_cast<size_t>(tb) * kTile * REC, tid, min(kTile, a.nj - tb * kTile) * REC);
  for (int tt = tb; tt < te; ++tt) {
    const int jbase = tt * kTile;
    const int cnt = min(kTile, a.nj - jbase);
    __syncthreads();
    nxt.store(tile, tid, cnt * REC);
    {
      const int tn = min(tt + 1, te - 1); // the last tile loads itself again
      nxt.load(jp + static_cast<size_t>(tn) * kTile * REC, tid, min(kTile, a.nj - tn * kTile) * REC);
    }
    __syncthreads();
    n.tile(tile, jbase, cnt, eps2, a.nb_count, a.nb_slot);
    // while the tile is still in LDS: the exact nearest neighbour so far
    // decides which groups of a ragged tile fold into float64 (fold_or_add),
    // as in force_fused and the batched kernel
    n.resolve(tile, jbase);
  }

  double bestd;
  int bslot;
  n.lane_sum(reinterpret_cast<double *>(lds), tid, il, ipw, bestd, bslot);
  if (n.sub == 0 && n.valid) {
    const size_t ni = static_cast<size_t>(a.ni);
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = n.t.acc[d];
      p[(3 + d) * ni] = n.t.jrk[d];
    }
    p[6 * ni] = n.t.pot;
    a.nn_r2[blockIdx.y * ni + i] = bestd;
    a.nn_slot[blockIdx.y * ni + i] = bslot;
  }
}

// ------------------------------------ small blocks, predictor fused in

// A block of at most 256 i-particles (one i-block, NarrowLane as in
// force_kernel) reads the float64 j-memory and predicts every tile into LDS
// itself (Sec. 2.2 fused into the tile load, as in the batched kernel), so
// the predicted records are never written to HBM and read back: for a block
// of a few particles the step is the predictor's HBM traffic, 112 B per
// j-particle instead of 112 + 48 + 48.  The next tile's j-memory entries are
// loaded into registers while the current tile is evaluated.  The
// neighbours are counted in nb_work, which the reduction clears again, so no
// launch before this one has to clear counters; workgroup (0, 0) clears the
// status words, which only the reduction after this launch writes.
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG) void force_fused(ForceArgs a, JMem jm, double ti, int *__restrict__ nb_work,
                                                   int *__restrict__ status) {
  constexpr int REC = rec4<PREC>();
  __shared__ __attribute__((aligned(16))) unsigned char lds[narrow_lds_bytes<PREC>()];
  float4 *tile = reinterpret_cast<float4 *>(lds);

  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid < kStatusWords) status[tid] = 0;
  const int ipw = a.ipw;
  const int il = tid & (ipw - 1);
  const int i = blockIdx.x * ipw + il;
  NarrowLane<PREC, NBL> n;
  n.init(a, i, i < a.ni, tid >> a.log2ipw, 8 - a.log2ipw);
  const real_t<PREC> eps2 = static_cast<real_t<PREC>>(a.eps2);

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int tb = blockIdx.y * per;
  const int te = min(ntiles, tb + per);

  // lane tid predicts record tid of each tile; past nj it loads slot nj - 1
  // (in bounds) and stores nothing
  JRaw nxt;
  if (tb < te) nxt.load(jm, static_cast<size_t>(min(tb * kTile + tid, a.nj - 1)));
  for (int tt = tb; tt < te; ++tt) {
    const int jbase = tt * kTile;
    const int cnt = min(kTile, a.nj - jbase);
    __syncthreads();
    if (tid < cnt) predict_raw<PREC>(nxt, ti, tile + tid * REC);
    if (tt + 1 < te) nxt.load(jm, static_cast<size_t>(min((tt + 1) * kTile + tid, a.nj - 1)));
    __syncthreads();
    n.tile(tile, jbase, cnt, eps2, nb_work, a.nb_slot);
    n.resolve(tile, jbase); // while the tile is still in LDS
  }

  double bestd;
  int bslot;
  n.lane_sum(reinterpret_cast<double *>(lds), tid, il, ipw, bestd, bslot);
  if (n.sub == 0 && n.valid) {
    const size_t ni = static_cast<size_t>(a.ni);
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = n.t.acc[d];
      p[(3 + d) * ni] = n.t.jrk[d];
    }
    p[6 * ni] = n.t.pot;
    a.nn_r2[blockIdx.y * ni + i] = bestd;
    a.nn_slot[blockIdx.y * ni + i] = bslot;
  }
}

// One i-particle (ipw = 1, all 256 lanes on it): lane tid takes records
// tid, tid + 256, ... of the split, predicts each one itself and uses it at
// once, so no record goes through LDS and no barrier is needed; the next
// record's j-memory entries are loaded while the current one is evaluated.
// The arithmetic and the order of the sums are those of force_fused (and of
// force_kernel on predicted records) for one i-particle: each record is a
// group of one pair, added to the float64 totals.
template <int PREC, bool NBL>
__global__ __launch_bounds__(kWG) void force_fused_one(ForceArgs a, JMem jm, double ti, int *__restrict__ nb_work,
                                                       int *__restrict__ status) {
  constexpr int REC = rec4<PREC>();
  __shared__ __attribute__((aligned(16))) double red[9 * kWG]; // lane_sum
  const int tid = threadIdx.x;
  if (blockIdx.y == 0 && tid < kStatusWords) status[tid] = 0;
  NarrowLane<PREC, NBL> n;
  n.init(a, 0, true, tid, 8);
  const real_t<PREC> eps2 = static_cast<real_t<PREC>>(a.eps2);

  const int ntiles = (a.nj + kTile - 1) / kTile;
  const int per = (ntiles + gridDim.y - 1) / gridDim.y;
  const int tb = blockIdx.y * per;
  const int te = min(ntiles, tb + per);
  const int je = min(a.nj, te * kTile);
  // kFusedDepth records per lane in flight: record js + u * kWG sits in q[u]
  // and is replaced, once used, by the one kFusedDepth records further on
  constexpr int D = kFusedDepth;
  JRaw q[D];
  const int j0 = tb * kTile + tid;
#pragma unroll
  for (int u = 0; u < D; ++u)
    if (j0 + u * kWG < je) q[u].load(jm, static_cast<size_t>(j0 + u * kWG));
  for (int js = j0; js < je; js += D * kWG) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int jj = js + u * kWG;
      if (jj < je) {
        float4 rec[REC];
        predict_raw<PREC>(q[u], ti, rec);
        if (jj + D * kWG < je) q[u].load(jm, static_cast<size_t>(jj + D * kWG));
        MaskedRun<PREC, NBL, false, true> run;
        run.start();
        run.step(n.st, n.ts, n.t, rec, jj, n.slot, eps2, n.h2, n.ebest, n.eslot, nb_work, a.nb_slot);
        run.finish(n.ts);
        fold(n.ts, n.t);
      }
    }
  }

  double bestd;
  int bslot;
  n.lane_sum(red, tid, 0, 1, bestd, bslot);
  if (tid == 0) {
    const size_t ni = static_cast<size_t>(a.ni);
    double *p = a.part + static_cast<size_t>(blockIdx.y) * 7 * ni;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      p[d * ni] = n.t.acc[d];
      p[(3 + d) * ni] = n.t.jrk[d];
    }
    p[6 * ni] = n.t.pot;
    a.nn_r2[blockIdx.y * ni] = bestd;
    a.nn_slot[blockIdx.y * ni] = bslot;
  }
}

// Clear n counters (a new or regrown nb_work buffer).
__global__ __launch_bounds__(256) void zero_kernel(int n, int *__restrict__ p) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < n) p[k] = 0;
}

// --------------------------------------------------------------- reduction

// 2^log2G lanes per i-particle (split_sum, then finish_out on the first
// lane), laid out by split_lane_map: float64 sum over the j-splits in a fixed
// order, nearest-neighbour minimum, neighbour-list finalisation.  The
// partials of position i belong to row iperm[i] when iperm is given (the
// spatially ordered kernel writes them in sorted order), else to row i.
// status[kStatusFlags] bit 0: a non-finite output; bit 1: a neighbour list
// overflowed (those i-particles are queued in ovf_list for nb_exact_kernel).
__global__ __launch_bounds__(256) void reduce_kernel(
    int nsplit, int ni, int log2G, const int *__restrict__ iperm, const double *__restrict__ part,
    const double *__restrict__ nn_r2, const int *__restrict__ nn_slot,
    const int *__restrict__ jindex, int *__restrict__ nb_count,
    int *__restrict__ nb_slot, int nbl, double *__restrict__ acc,
    double *__restrict__ jerk, double *__restrict__ pot, int *__restrict__ nnb,
    double *__restrict__ r2nn, int *__restrict__ status, int *__restrict__ ovf_list,
    int *__restrict__ nb_work) {
  const long long t = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
  const int G = 1 << log2G;
  int ioff, g, xs;
  split_lane_map(static_cast<int>(t & 63), G, ioff, g, xs);
  const long long i = (t >> 6) * xs + ioff;
  if (i >= ni) return; // whole groups: the G lanes of an i-particle share i
  const size_t n = static_cast<size_t>(ni);
  double sum[7], best;
  int bslot;
  split_sum(nsplit, G, g, xs, part + i, 7 * n, n, nn_r2 + i, nn_slot + i, n, sum, best, bslot);
  if (g != 0) return;
  const int row = iperm ? iperm[i] : static_cast<int>(i);
  const int fl = finish_out(sum, best, bslot, row, jindex, nb_count, nb_slot, nbl != 0, acc, jerk, pot, nnb, r2nn,
                            status, ovf_list, nullptr, 0, nb_work);
  if (fl) atomicOr(status + kStatusFlags, fl);
}

// A block of few i-particles over many j-splits: one workgroup per
// i-particle.  Lane g adds splits g, g + 256, ... in float64 (all of its
// loads issued before the additions), the 64 lane sums of a wave meet in an
// xor butterfly, and lane 0 adds the four wave sums in wave order: the order
// of additions is fixed by nsplit alone.  The 64 lanes per particle of
// reduce_kernel need two or more rounds of dependent loads for 512 splits
// and occupy a handful of workgroups; here each lane's loads are one round.
__global__ __launch_bounds__(256) void reduce_few_kernel(
    int nsplit, int ni, const int *__restrict__ iperm, const double *__restrict__ part,
    const double *__restrict__ nn_r2, const int *__restrict__ nn_slot,
    const int *__restrict__ jindex, int *__restrict__ nb_count,
    int *__restrict__ nb_slot, int nbl, double *__restrict__ acc,
    double *__restrict__ jerk, double *__restrict__ pot, int *__restrict__ nnb,
    double *__restrict__ r2nn, int *__restrict__ status, int *__restrict__ ovf_list,
    int *__restrict__ nb_work) {
  constexpr int kPer = kFewSplitsPerLane;
  const int i = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t n = static_cast<size_t>(ni);
  double v[kPer][7], r2[kPer];
  int sl[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = tid + u * 256;
    const bool ok = q < nsplit;
    const size_t k = static_cast<size_t>(ok ? q : 0);
#pragma unroll
    for (int c = 0; c < 7; ++c) v[u][c] = ok ? part[k * 7 * n + c * n + i] : 0.0;
    r2[u] = ok ? nn_r2[k * n + i] : INFINITY;
    sl[u] = ok ? nn_slot[k * n + i] : -1;
  }
  double s[7], best = INFINITY;
  int bslot = -1;
#pragma unroll
  for (int c = 0; c < 7; ++c) s[c] = 0.0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += v[u][c];
    nn_merge(r2[u], sl[u], best, bslot);
  }
  for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += __shfl_xor(s[c], m);
    const double ob = __shfl_xor(best, m);
    const int os = __shfl_xor(bslot, m);
    nn_merge(ob, os, best, bslot);
  }
  __shared__ double s_red[4][8];
  __shared__ int s_slot[4];
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s_red[wave][c] = s[c];
    s_red[wave][7] = best;
    s_slot[wave] = bslot;
  }
  __syncthreads();
  if (tid != 0) return;
#pragma unroll
  for (int w = 1; w < 4; ++w) {
#pragma unroll
    for (int c = 0; c < 7; ++c) s[c] += s_red[w][c];
    nn_merge(s_red[w][7], s_slot[w], best, bslot);
  }
  const int row = iperm ? iperm[i] : i;
  const int fl = finish_out(s, best, bslot, row, jindex, nb_count, nb_slot, nbl != 0, acc, jerk, pot, nnb, r2nn,
                            status, ovf_list, nullptr, 0, nb_work);
  if (fl) atomicOr(status + kStatusFlags, fl);
}

// --------------------------------------------- neighbour-list overflow

// One workgroup per queued i-particle (grid-strided over the queue): its
// list rebuilt by exact_list over slots 0 .. nj - 1 of the predicted records.
template <int PREC>
__global__ __launch_bounds__(kWG) void nb_exact_kernel(ForceArgs a, const int *__restrict__ jindex,
                                                        const int *__restrict__ status,
                                                        const int *__restrict__ ovf_list) {
  constexpr int REC = rec4<PREC>();
  __shared__ unsigned s_cnt;
  __shared__ int s_keep[kNbMax];
  const float4 *jp = static_cast<const float4 *>(a.jpred);
  auto rec_of = [jp](int js, float4 *) { return jp + static_cast<size_t>(js) * REC; };
  const int novf = status[kStatusOverflowCount];
  for (int q = blockIdx.x; q < novf; q += gridDim.x) {
    const int i = ovf_list[q];
    IState<PREC> st;
    int slot;
    real_t<PREC> h2;
    load_i<PREC>(st, a, i, true, slot, h2);
    exact_list<PREC>(st, slot, h2, 0, a.nj, jindex, rec_of, a.nb_slot + static_cast<size_t>(i) * kNbMax,
                     a.nb_count + i, s_cnt, s_keep);
  }
}

// The same for a calculation of force_fused, which kept no predicted
// records: each record is predicted again from the j-memory exactly as in
// force_fused.
template <int PREC>
__global__ __launch_bounds__(kWG) void nb_exact_fused_kernel(ForceArgs a, JMem jm, double ti,
                                                              const int *__restrict__ status,
                                                              const int *__restrict__ ovf_list) {
  __shared__ unsigned s_cnt;
  __shared__ int s_keep[kNbMax];
  auto rec_of = [jm, ti](int js, float4 *buf) -> const float4 * {
    predict_record<PREC>(jm, static_cast<size_t>(js), ti, buf);
    return buf;
  };
  const int novf = status[kStatusOverflowCount];
  for (int q = blockIdx.x; q < novf; q += gridDim.x) {
    const int i = ovf_list[q];
    IState<PREC> st;
    int slot;
    real_t<PREC> h2;
    load_i<PREC>(st, a, i, true, slot, h2);
    exact_list<PREC>(st, slot, h2, 0, a.nj, jm.index, rec_of, a.nb_slot + static_cast<size_t>(i) * kNbMax,
                     a.nb_count + i, s_cnt, s_keep);
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

// ------------------------------------------------------ static scratch

// Work buffers of g6mi_calc_device_noalloc (callers that cannot allocate):
// one array of G6MI_NOALLOC_SCRATCH_BYTES in each GPU's memory, held from
// the library's load on that GPU until the process ends.  In host code the
// name stands for no device address: only the address that
// hipGetSymbolAddress returns for the current device is used.
static __device__ __align__(256) unsigned char scratch[G6MI_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_region(int device, void **ptr, size_t *bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    // once per device, with that device current
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  *bytes = sizeof(scratch);
  return hipSuccess;
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
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP32>, grid, block, 0, s, nj, ti, jm, out, nb_count,
                       ni, status);
    break;
  case G6MI_PREC_DS:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_DS>, grid, block, 0, s, nj, ti, jm, out, nb_count,
                       ni, status);
    break;
  default:
    hipLaunchKernelGGL(predict_kernel<G6MI_PREC_FP64>, grid, block, 0, s, nj, ti, jm, out, nb_count,
                       ni, status);
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

template <int PREC>
static void launch_fused_prec(bool nbl, const ForceArgs &a, const JMem &jm, double ti, int *nb_work, int *status,
                              dim3 grid, hipStream_t s) {
  if (a.ipw == 1) {
    if (nbl)
      hipLaunchKernelGGL((force_fused_one<PREC, true>), grid, dim3(kWG), 0, s, a, jm, ti, nb_work, status);
    else
      hipLaunchKernelGGL((force_fused_one<PREC, false>), grid, dim3(kWG), 0, s, a, jm, ti, nb_work, status);
    return;
  }
  if (nbl)
    hipLaunchKernelGGL((force_fused<PREC, true>), grid, dim3(kWG), 0, s, a, jm, ti, nb_work, status);
  else
    hipLaunchKernelGGL((force_fused<PREC, false>), grid, dim3(kWG), 0, s, a, jm, ti, nb_work, status);
}

hipError_t launch_force_fused(int prec, bool nbl, const ForceArgs &a, const JMem &jm, double ti, int *nb_work,
                              int *status, int nsplit, hipStream_t s) {
  if (a.ni <= 0 || a.ipw > kWG) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>((a.ni + a.ipw - 1) / a.ipw), static_cast<unsigned>(nsplit));
  switch (prec) {
  case G6MI_PREC_FP32: launch_fused_prec<G6MI_PREC_FP32>(nbl, a, jm, ti, nb_work, status, grid, s); break;
  case G6MI_PREC_DS: launch_fused_prec<G6MI_PREC_DS>(nbl, a, jm, ti, nb_work, status, grid, s); break;
  default: launch_fused_prec<G6MI_PREC_FP64>(nbl, a, jm, ti, nb_work, status, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_zero(int n, int *p, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, p);
  return hipGetLastError();
}

hipError_t launch_reduce(int nsplit, int ni, const int *iperm, const double *part, const double *nn_r2,
                         const int *nn_slot, const int *jindex, int *nb_count, int *nb_slot,
                         bool nbl, double *acc, double *jerk, double *pot, int *nnb,
                         double *r2nn, int *status, int *ovf_list, hipStream_t s, int *nb_work) {
  if (ni <= 0) return hipSuccess;
  if (ni <= kFewMaxNi && nsplit > 64 && nsplit <= 256 * kFewSplitsPerLane) {
    hipLaunchKernelGGL(reduce_few_kernel, dim3(static_cast<unsigned>(ni)), dim3(256), 0, s, nsplit, ni, iperm, part,
                       nn_r2, nn_slot, jindex, nb_count, nb_slot, nbl ? 1 : 0, acc, jerk, pot, nnb, r2nn, status,
                       ovf_list, nb_work);
    return hipGetLastError();
  }
  const int G = split_lanes(nsplit, ni);
  int log2G = 0;
  while ((1 << log2G) < G) ++log2G;
  const long long waves = (ni + (64 >> log2G) - 1) / (64 >> log2G);
  const long long lanes = waves * 64;
  hipLaunchKernelGGL(reduce_kernel, dim3(static_cast<unsigned>((lanes + 255) / 256)), dim3(256), 0, s, nsplit, ni,
                     log2G, iperm, part, nn_r2, nn_slot, jindex, nb_count, nb_slot, nbl ? 1 : 0, acc, jerk, pot,
                     nnb, r2nn, status, ovf_list, nb_work);
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

hipError_t launch_nb_exact_fused(int prec, const ForceArgs &a, const JMem &jm, double ti, const int *status,
                                 const int *ovf_list, int novf, hipStream_t s) {
  if (novf <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(novf < 1024 ? novf : 1024));
  switch (prec) {
  case G6MI_PREC_FP32:
    hipLaunchKernelGGL(nb_exact_fused_kernel<G6MI_PREC_FP32>, grid, dim3(kWG), 0, s, a, jm, ti, status, ovf_list);
    break;
  case G6MI_PREC_DS:
    hipLaunchKernelGGL(nb_exact_fused_kernel<G6MI_PREC_DS>, grid, dim3(kWG), 0, s, a, jm, ti, status, ovf_list);
    break;
  default:
    hipLaunchKernelGGL(nb_exact_fused_kernel<G6MI_PREC_FP64>, grid, dim3(kWG), 0, s, a, jm, ti, status, ovf_list);
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
