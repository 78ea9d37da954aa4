// Device pieces of the batched launch shared by the batch kernels
// (g6mi_batch.hip) and the device-resident block steps (g6mi_hermite.hip):
// the per-cluster launch plan and the reduction of one i-block's split
// partials.  The plan functions also compile for the host, where a test
// checks their invariants.

#pragma once

#include "g6mi_device.h"

namespace g6mi {

// Block shape of a cluster of ni i-particles against nj j-slots: two
// i-particles per lane from wide_min on, else the next power of two up to
// 256 and up to the item target (item_work * 128 lane-pairs, not below
// kBatchMinIpw), so that one tile of a narrow block stays within the target.
// The tile count is kept in per until the splits are chosen.
__host__ __device__ __forceinline__ BatchPlan plan_shape(int ni, int nj, const BatchTune &t) {
  BatchPlan pl{};
  int ipw = 1, l2 = 0;
  if (ni >= t.wide_min) {
    ipw = 2 * kWG;
    l2 = 9;
  } else {
    const long long cap = max(static_cast<long long>(kBatchMinIpw), static_cast<long long>(t.item_work) * 128);
    while (ipw < ni && ipw < kWG && 2 * ipw <= cap) {
      ipw <<= 1;
      ++l2;
    }
  }
  pl.ipw = ipw;
  pl.log2ipw = l2;
  pl.nib = ni > 0 ? (ni + ipw - 1) / ipw : 0;
  pl.per = (nj + kTile - 1) / kTile;
  pl.ni = ni;
  return pl;
}

// Lane-pairs of a shaped cluster (one tile costs a lane ipw pairs on a
// narrow block, 512 on a wide one).
__host__ __device__ __forceinline__ long long plan_work(const BatchPlan &pl) {
  return static_cast<long long>(pl.nib) * pl.per * pl.ipw;
}

// A cluster whose i-blocks cannot make `share` items even with the most
// splits (one tile each, at most max_split) takes smaller i-blocks, down to
// kBatchMinIpw, with more lanes per i-particle: a lone block of 340 against
// 32768 particles then runs as 11 blocks of 32 in 704 items instead of 2
// blocks of 256 in 128 items.  Returns whether the shape changed.
__host__ __device__ __forceinline__ bool plan_share(BatchPlan &pl, long long share, const BatchTune &t) {
  const int most = min(max(pl.per, 1), t.max_split);
  if (pl.nib == 0 || static_cast<long long>(pl.nib) * most >= share) return false;
  while (pl.ipw > kBatchMinIpw && static_cast<long long>(pl.nib) * most < share) {
    pl.ipw = min(pl.ipw >> 1, kWG);
    pl.log2ipw = __builtin_ctz(pl.ipw);
    pl.nib = (pl.ni + pl.ipw - 1) / pl.ipw;
  }
  return true;
}

// Item target in lane-pairs: item_work * 128, lowered (down to one) until
// the batch's work makes about one item per persistent workgroup.
__host__ __device__ __forceinline__ long long plan_target(long long work, int grid, const BatchTune &t) {
  return max(1LL, min(static_cast<long long>(t.item_work) * 128, work / max(1, grid)));
}

// Tiles per split and split count of a shaped cluster for the item target,
// at most max_split splits.
__host__ __device__ __forceinline__ void plan_splits(BatchPlan &pl, long long target, const BatchTune &t) {
  const int ntiles = pl.per;
  int per = static_cast<int>(max(1LL, min(static_cast<long long>(max(ntiles, 1)), target / pl.ipw)));
  int nsplit = ntiles > 0 ? (ntiles + per - 1) / per : 1;
  if (nsplit > t.max_split) {
    per = (ntiles + t.max_split - 1) / t.max_split;
    nsplit = (ntiles + per - 1) / per;
  }
  pl.per = per;
  pl.nsplit = nsplit;
}

// Queue class of a shaped cluster's items: the item table lists class 0,
// then 1, then 2, each in cluster order, and the persistent workgroups take
// items in table order.  Class 0: narrow blocks of fewer than 64
// i-particles, whose items run several tiles, each a round trip to memory
// with little arithmetic behind it (long in time, light on the VALU: they
// run best beside computing items, from the start).  Class 1: wide blocks,
// the longest computing items.  Class 2: the other narrow blocks, whose
// items (one or two tiles) are the shortest and fill the end of the launch.
// Queued in cluster order, the last items were whichever wide blocks came
// last, and a third of the workgroups idled through the final round.
constexpr int kItemOrders = 3;
__host__ __device__ __forceinline__ int plan_order(const BatchPlan &pl) {
  return pl.ipw == 2 * kWG ? 1 : (pl.ipw < 64 ? 0 : 2);
}

// Parts per i-block of a batch reduction over nib i-blocks on a grid of
// `grid` workgroups: the largest power of two up to `cap` (and 64) that
// still gives every (i-block, part) a workgroup of its own, else 1 (the
// grid strides over whole i-blocks).  A part is a contiguous run of the
// i-block's rows; more parts put more workgroups, and so more loads in
// flight, on the split partials, whose long sums are bound by latency.
__host__ __device__ __forceinline__ int reduce_parts(int nib, int grid, int cap) {
  int P = 1;
  while (2 * P <= min(cap, 64) && static_cast<long long>(nib) * (2 * P) <= grid) P <<= 1;
  return P;
}

// The float64 sum of the split partials (split_sum, G lanes per i-particle
// as the splits and the workgroup allow, laid out by split_lane_map) of part
// `part` of `nparts` of i-block ibg, and its rows' results (finish_out).
// The part holds ipw / P consecutive rows, P = min(nparts, ipw) (both powers
// of two); parts from P on are empty.  Every thread of the workgroup calls
// it with the same arguments; epi(row, sum) runs on the lane that wrote row
// `row`, after the write, with the row's sums (acc xyz, jerk xyz, sum m/r).
// ONE: the batch is one cluster (cluster 0), whose i-block table need not be
// read.  Returns the status flags of this thread's rows.
template <bool ONE = false, class Epi>
__device__ __forceinline__ int reduce_iblock(const BatchArgs &b, int ibg, int part, int nparts, Epi &&epi) {
  const int tid = threadIdx.x;
  const int c = ONE ? 0 : __builtin_amdgcn_readfirstlane(b.ib_cl[ibg]);
  const g6mi_cluster d = b.cl[c];
  const BatchPlan p = b.plan[c];
  const int ib = ibg - p.ib0;
  const int P = min(nparts, p.ipw);
  if (part >= P) return 0;
  const int rows = p.ipw / P;
  const int G = min(split_lanes(p.nsplit, 1), max(1, kWG / rows));
  int ioff, g, xs;
  split_lane_map(tid & 63, G, ioff, g, xs);
  int fl = 0;
  for (int k0 = 0; k0 < rows; k0 += kWG / G) {
    const int kk = k0 + (tid >> 6) * xs + ioff;
    const int il = ib * p.ipw + part * rows + kk;
    if (kk < rows && il < d.ni) {
      const size_t e = static_cast<size_t>(p.pbase) + il;
      double sum[7], best;
      int bslot;
      split_sum(p.nsplit, G, g, xs, b.part + e, static_cast<size_t>(d.ni), b.pcap, b.nn_r2 + e, b.nn_slot + e,
                static_cast<size_t>(d.ni), sum, best, bslot);
      if (g == 0) {
        fl |= finish_out(sum, best, bslot, d.ioff + il, b.jm.index, b.fa.nb_count, b.fa.nb_slot, b.nbl != 0, b.acc,
                         b.jerk, b.pot, b.nnb, b.r2nn, b.status, b.ovf_list, b.ovf_tag, c);
        epi(d.ioff + il, static_cast<const double *>(sum));
      }
    }
  }
  return fl;
}

} // namespace g6mi
