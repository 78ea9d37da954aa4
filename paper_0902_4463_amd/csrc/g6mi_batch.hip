// Batched multi-cluster force evaluation: many independent systems of
// uneven size and uneven active blocks in one launch.
//
//   batch_plan_kernel  -- one workgroup turns the cluster descriptors into a
//                         per-cluster launch plan (i-particles per workgroup,
//                         j-splits) and a flat list of work items
//                         (cluster, i-block, j-split); the other workgroups
//                         clear the per-row counters of the calculation.
//   batch_kernel       -- persistent workgroups take items from work queues
//                         (a static first round, then eight atomic counters).
//                         An item predicts its j-tiles
//                         straight into LDS from the float64 j-memory (the
//                         predictor of Sec. 2.2 fused into the tile load),
//                         runs the interaction of Sec. 2.3 on them and stores
//                         its split partials.
//   batch_reduce       -- workgroups over parts of the i-blocks add the
//                         partials of all splits in a fixed order and write
//                         the results (the reduction of Sec. 2.3).
//   batch_nb_exact     -- exact neighbour lists for overflowed i-particles.
//
// Each cluster is what the paper's library evaluates per call; batching them
// fills the 256 compute units when every single cluster is far too small to
// do so, and removes the per-call launches.

#include "g6mi_batch_common.h"

namespace g6mi {

// -------------------------------------------------------------------- plan

// Inclusive sum of x over the 256 threads of a workgroup (wave shuffles, then
// the four wave totals through LDS); all = the workgroup total.  Every
// thread must call it; it ends with a barrier, so s_part can be reused.
template <class T> __device__ __forceinline__ T wg_scan(T x, T *s_part, T &all) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_part[wave] = x;
  __syncthreads();
  T base = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const T p = s_part[w];
    if (w < wave) base += p;
    sum += p;
  }
  __syncthreads();
  all = sum;
  return x + base;
}

// Index of the first of 256 non-decreasing counts above q (one exists).
__device__ __forceinline__ int first_above(const int *inc, int q) {
  int lo = 0, hi = 255;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (inc[mid] > q) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Work items: for cluster c with ni i-particles in nib i-blocks of ipw and
// ntiles j-tiles in nsplit splits of `per` tiles, nib * nsplit items.  One
// tile costs a lane ipw pairs (narrow blocks) or 512 (wide blocks).  Items
// cost about the same: per = target / ipw tiles, where the target is
// item_work * 128 lane-pairs, lowered (down to one tile) until the whole
// batch makes at least about one item per persistent workgroup, so that a
// batch of few or small clusters still spreads over the GPU.  A narrow
// block holds at most the target's worth of i-particles (not below
// kBatchMinIpw), so that one tile of it stays within the target.
//
// Pass 1 checks the descriptors, picks the block shape of each cluster
// (kept in its plan entry) and adds up the batch's work; pass 1b cuts the
// blocks of clusters too small to fill their share of the GPU; pass 2 picks
// the splits, scans i-blocks and partial entries and fills the i-block ->
// cluster table; pass 3 scans the items class by class (plan_order) and
// fills the item -> cluster table.
__global__ __launch_bounds__(256) void batch_plan_kernel(BatchArgs b) {
  const int tid = threadIdx.x;
  if (blockIdx.x > 0) {
    // rows (blockIdx.x - 1) * chunk ...: neighbour counts
    const int base = (blockIdx.x - 1) * kPlanZeroChunk;
    if (b.nbl)
      for (int k = tid; k < kPlanZeroChunk; k += 256) {
        const int r = base + k;
        if (r < b.ni_total) b.fa.nb_count[r] = 0;
      }
    return;
  }
  __shared__ long long s_part[4];
  __shared__ int s_inc[256], s_inc_ib[256];
  __shared__ int s_flags;
  if (tid == 0) s_flags = 0;
  __syncthreads();

  // With one chunk (ncl <= 256) each thread keeps its cluster's entry in
  // registers from pass to pass (pl_last), instead of a round trip through
  // memory per pass; with more, it reads back its own entry of each chunk.
  BatchPlan pl_last{};
  const bool one_chunk = b.ncl <= 256;

  // pass 1: validity, block shape, work
  long long c_rows = 0, work = 0;
  for (int c0 = 0; c0 < b.ncl; c0 += 256) {
    const int c = c0 + tid;
    int ni = 0, nj = 0;
    bool ok = false;
    if (c < b.ncl) {
      const g6mi_cluster d = b.cl[c];
      ok = d.joff >= 0 && d.nj >= 0 && static_cast<long long>(d.joff) + d.nj <= b.nj_set && d.ioff >= 0 &&
           d.ni >= 0 && static_cast<long long>(d.ioff) + d.ni <= b.ni_total && isfinite(d.ti) &&
           isfinite(d.eps2) && d.eps2 >= 0.0;
      ni = ok ? d.ni : 0;
      nj = ok ? d.nj : 0;
    }
    // Clusters sharing i-rows could add up to more rows than ni_total, and
    // the i-block counters and partial sums are sized by ni_total: every
    // cluster past that many rows in total is skipped.
    long long rows_all;
    const long long rows = wg_scan<long long>(ni, s_part, rows_all);
    if (ok && c_rows + rows > b.ni_total) {
      ok = false;
      ni = nj = 0;
    }
    if (c < b.ncl && !ok) atomicOr(&s_flags, kFlagBadCluster);
    const BatchPlan pl = plan_shape(ni, nj, b.tune); // splits in pass 2
    if (c < b.ncl) b.plan[c] = pl;
    pl_last = pl;
    long long work_all;
    wg_scan<long long>(plan_work(pl), s_part, work_all);
    work += work_all;
    c_rows += rows_all;
  }
  // pass 1b: clusters too small for their share of the persistent
  // workgroups (plan_share); the share is the grid times the cluster's
  // fraction of the batch's work
  const long long work0 = max(1LL, work);
  work = 0;
  for (int c0 = 0; c0 < b.ncl; c0 += 256) {
    const int c = c0 + tid;
    long long w = 0;
    if (c < b.ncl) {
      BatchPlan pl = one_chunk ? pl_last : b.plan[c];
      if (pl.nib > 0) {
        const long long share = (static_cast<long long>(b.grid) * plan_work(pl) + work0 - 1) / work0;
        if (plan_share(pl, share, b.tune)) b.plan[c] = pl;
        w = plan_work(pl);
      }
      pl_last = pl;
    }
    long long work_all;
    wg_scan<long long>(w, s_part, work_all);
    work += work_all;
  }
  const long long target = plan_target(work, b.grid, b.tune);

  // pass 2: splits, the i-block and partial-entry scans in cluster order
  // (each thread reads back its own pass-1 entries) and the i-block ->
  // cluster table, filled by all threads: i-block q of the chunk belongs to
  // the first cluster whose inclusive i-block count exceeds q
  int c_nib = 0;
  long long c_pent = 0;
  for (int c0 = 0; c0 < b.ncl; c0 += 256) {
    const int c = c0 + tid;
    int nib = 0, ni = 0, nsplit = 1;
    BatchPlan pl{};
    if (c < b.ncl) {
      pl = one_chunk ? pl_last : b.plan[c];
      plan_splits(pl, target, b.tune);
      nib = pl.nib;
      ni = pl.ni;
      nsplit = pl.nsplit;
    }
    const long long pent = static_cast<long long>(ni) * nsplit;
    long long nib_all, pent_all;
    const int nibs = static_cast<int>(wg_scan<long long>(nib, s_part, nib_all));
    const long long pents = wg_scan<long long>(pent, s_part, pent_all);
    if (c < b.ncl) {
      pl.ib0 = c_nib + nibs - nib;
      pl.pbase = c_pent + pents - pent;
      b.plan[c] = pl;
    }
    pl_last = pl;
    s_inc_ib[tid] = nibs;
    __syncthreads();
    for (int q = tid; q < nib_all; q += 256) b.ib_cl[c_nib + q] = c0 + first_above(s_inc_ib, q);
    __syncthreads(); // s_inc_ib is rewritten by the next chunk
    c_nib += static_cast<int>(nib_all);
    c_pent += pent_all;
  }
  // pass 3: the item scan and the item -> cluster table, one queue class
  // (plan_order) after the other, in cluster order within a class
  int c_items = 0;
  for (int k = 0; k < kItemOrders; ++k) {
    for (int c0 = 0; c0 < b.ncl; c0 += 256) {
      const int c = c0 + tid;
      long long n = 0;
      if (c < b.ncl) {
        const BatchPlan pl = one_chunk ? pl_last : b.plan[c];
        if (plan_order(pl) == k) n = static_cast<long long>(pl.nib) * pl.nsplit;
      }
      long long items_all;
      const int items = static_cast<int>(wg_scan<long long>(n, s_part, items_all));
      if (n > 0) b.plan[c].item0 = c_items + items - static_cast<int>(n);
      s_inc[tid] = items;
      __syncthreads();
      for (int q = tid; q < items_all; q += 256)
        if (c_items + q < b.item_cap) b.item_cl[c_items + q] = c0 + first_above(s_inc, q);
      __syncthreads(); // s_inc is rewritten by the next chunk
      c_items += static_cast<int>(items_all);
    }
  }
  if (tid == 0) {
    for (int x = 0; x < kQueues; ++x) b.work->head[x] = 0;
    b.work->nitems = min(c_items, b.item_cap);
    b.work->nib = c_nib;
    // more items than the table holds cannot happen with the host's bound;
    // it would drop work, so it is reported like a bad descriptor
    b.status[kStatusFlags] = s_flags | (c_items > b.item_cap ? kFlagBadCluster : 0);
    b.status[kStatusOverflowCount] = 0;
  }
}

// ------------------------------------------------------ persistent kernel

__device__ __forceinline__ void store_partial(const BatchArgs &b, size_t e, const Totals &t, double best,
                                              int bslot) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b.part[d * b.pcap + e] = t.acc[d];
    b.part[(3 + d) * b.pcap + e] = t.jrk[d];
  }
  b.part[6 * b.pcap + e] = t.pot;
  b.nn_r2[e] = best;
  b.nn_slot[e] = bslot;
}

// Persistent workgroups: workgroup g starts with item g, then takes the
// next item from its queue until the items run out (every wave reaches the
// exit: items are finite and each workgroup takes one item per round).  The
// items after the first grid's worth are dealt round-robin to kQueues
// queues, one counter each, and workgroup g takes from queue g mod kQueues:
// workgroups go to the 8 XCDs round-robin, so each XCD's workgroups share
// one counter, and no counter serves the whole grid.  The first round needs
// no atomic at all: hundreds of workgroups incrementing one counter at once
// queue up behind each other.
// Partial entry of i-particle il (cluster row) in split s: pbase + s * ni +
// il, component-major over pcap entries.
// WIDE = false: the narrow-only kernel, for batches whose plan cannot make a
// wide block (the host launches it only when tune.wide_min > ni_total); its
// registers fit four waves per SIMD.
template <int PREC, bool NBL, bool WIDE>
__global__ __launch_bounds__(kWG, WIDE ? wide_waves<PREC>() : kNarrowWaves) void batch_kernel(BatchArgs b) {
  using R = real_t<PREC>;
  constexpr int REC = rec4<PREC>();
  __shared__ __attribute__((aligned(16))) unsigned char lds[narrow_lds_bytes<PREC>()];
  __shared__ int s_item;
  float4 *tile = reinterpret_cast<float4 *>(lds);
  const int tid = threadIdx.x;
  const int nitems = b.work->nitems;

  for (int q = blockIdx.x; q < nitems;) {
    // q is uniform across the workgroup: the item's cluster, descriptor and
    // plan are then scalar loads held in scalar registers
    const int c = b.item_cl[q];
    const g6mi_cluster d = b.cl[c];
    const BatchPlan p = b.plan[c];
    const int r = q - p.item0;
    const int ib = r / p.nsplit;
    const int sp = r - ib * p.nsplit;
    const int ntiles = (d.nj + kTile - 1) / kTile;
    const int tb = sp * p.per;
    const int te = min(ntiles, tb + p.per);
    const int jend = d.joff + d.nj;
    const R eps2 = static_cast<R>(d.eps2);
    const size_t e0 = static_cast<size_t>(p.pbase) + static_cast<size_t>(sp) * d.ni;

    if (!WIDE && p.ipw > kWG) {
      // not reached (see above); the item is dropped and the batch flagged
      if (tid == 0) atomicOr(b.status + kStatusFlags, kFlagBadCluster);
    } else if (WIDE && p.ipw == 2 * kWG) {
      const int il0 = ib * (2 * kWG) + tid, il1 = il0 + kWG;
      WideLanes<PREC, NBL> w;
      w.init(b.fa, d.ioff + il0, d.ioff + il1, il0 < d.ni, il1 < d.ni);
      for (int tt = tb; tt < te; ++tt) {
        const int jbase = d.joff + tt * kTile;
        const int cnt = min(kTile, jend - jbase);
        __syncthreads();
        if (tid < cnt) predict_record<PREC>(b.jm, static_cast<size_t>(jbase + tid), d.ti, tile + tid * REC);
        __syncthreads();
        // DS: every group goes straight to the float64 totals (see WideLanes::tile)
        w.template tile<PREC == G6MI_PREC_DS, true>(tile, jbase, cnt, eps2, b.fa.nb_count, b.fa.nb_slot);
        w.resolve(tile, jbase); // while the tile is still in LDS
      }
      if (w.v0) store_partial(b, e0 + il0, w.t0, static_cast<double>(w.ebest0), w.eslot0);
      if (w.v1) store_partial(b, e0 + il1, w.t1, static_cast<double>(w.ebest1), w.eslot1);
    } else {
      const int ipw = p.ipw;
      const int lil = tid & (ipw - 1);
      const int il = ib * ipw + lil;
      NarrowLane<PREC, NBL> n;
      n.init(b.fa, d.ioff + il, il < d.ni, tid >> p.log2ipw, 8 - p.log2ipw);
      for (int tt = tb; tt < te; ++tt) {
        const int jbase = d.joff + tt * kTile;
        const int cnt = min(kTile, jend - jbase);
        __syncthreads();
        if (tid < cnt) predict_record<PREC>(b.jm, static_cast<size_t>(jbase + tid), d.ti, tile + tid * REC);
        __syncthreads();
        n.tile(tile, jbase, cnt, eps2, b.fa.nb_count, b.fa.nb_slot);
        n.resolve(tile, jbase);
      }
      double bestd;
      int bslot;
      n.lane_sum(reinterpret_cast<double *>(lds), tid, lil, ipw, bestd, bslot);
      if (n.sub == 0 && n.valid) store_partial(b, e0 + il, n.t, bestd, bslot);
    }
    if (static_cast<int>(gridDim.x) >= nitems) break; // no second round
    __syncthreads(); // the item is done with the LDS and s_item
    if (tid == 0) {
      // every queue needs a workgroup: one queue for a grid smaller than kQueues
      const int nq = static_cast<int>(gridDim.x) >= kQueues ? kQueues : 1;
      const int x = static_cast<int>(blockIdx.x) % nq;
      s_item = static_cast<int>(gridDim.x) + x + nq * atomicAdd(&b.work->head[x], 1);
    }
    __syncthreads();
    q = __builtin_amdgcn_readfirstlane(s_item);
  }
}

// One workgroup per part of an i-block (reduce_parts; grid-strided over the
// work->nib i-blocks of the batch when they outnumber the grid, ib_cl giving
// each one's cluster): the float64 sum of the rows' split partials
// (split_sum, G lanes per i-particle as the splits and the workgroup allow)
// and their results (finish_out).  A launch of its own: the kernel boundary
// makes every item's partials visible, where a release fence per item would
// write back the XCD's whole L2 (buffer_wbl2) and an acquire invalidate it,
// once per item.
__global__ __launch_bounds__(kWG) void batch_reduce_kernel(BatchArgs b) {
  const int nib_total = b.work->nib;
  const int P = reduce_parts(nib_total, static_cast<int>(gridDim.x), 64);
  int fl = 0;
  for (int u = blockIdx.x; u < nib_total * P; u += gridDim.x)
    fl |= reduce_iblock(b, u / P, u % P, P, [](int, const double *) {});
  if (fl) atomicOr(b.status + kStatusFlags, fl);
}

// ------------------------------------------------- neighbour-list overflow

// One workgroup per queued i-particle: its list rebuilt from the slots of
// its own cluster, each record predicted again exactly as in batch_kernel.
template <int PREC>
__global__ __launch_bounds__(kWG) void batch_nb_exact_kernel(BatchArgs b) {
  __shared__ unsigned s_cnt;
  __shared__ int s_keep[kNbMax];
  const int novf = b.status[kStatusOverflowCount];
  for (int q = blockIdx.x; q < novf; q += gridDim.x) {
    const int row = b.ovf_list[q];
    const g6mi_cluster d = b.cl[b.ovf_tag[q]];
    IState<PREC> st;
    int slot;
    real_t<PREC> h2;
    load_i<PREC>(st, b.fa, row, true, slot, h2);
    const JMem jm = b.jm;
    const double ti = d.ti;
    auto rec_of = [jm, ti](int js, float4 *buf) -> const float4 * {
      predict_record<PREC>(jm, static_cast<size_t>(js), ti, buf);
      return buf;
    };
    exact_list<PREC>(st, slot, h2, d.joff, d.joff + d.nj, jm.index, rec_of,
                     b.fa.nb_slot + static_cast<size_t>(row) * kNbMax, b.fa.nb_count + row, s_cnt, s_keep);
  }
}

// ---------------------------------------------------------------- launchers

hipError_t launch_batch_plan(const BatchArgs &b, hipStream_t s) {
  const unsigned zero_blocks = static_cast<unsigned>((b.ni_total + kPlanZeroChunk - 1) / kPlanZeroChunk);
  hipLaunchKernelGGL(batch_plan_kernel, dim3(1 + zero_blocks), dim3(256), 0, s, b);
  return hipGetLastError();
}

template <int PREC>
static void launch_batch_prec(const BatchArgs &b, int grid, hipStream_t s) {
  if (b.wide) {
    if (b.nbl)
      hipLaunchKernelGGL((batch_kernel<PREC, true, true>), dim3(grid), dim3(kWG), 0, s, b);
    else
      hipLaunchKernelGGL((batch_kernel<PREC, false, true>), dim3(grid), dim3(kWG), 0, s, b);
  } else {
    if (b.nbl)
      hipLaunchKernelGGL((batch_kernel<PREC, true, false>), dim3(grid), dim3(kWG), 0, s, b);
    else
      hipLaunchKernelGGL((batch_kernel<PREC, false, false>), dim3(grid), dim3(kWG), 0, s, b);
  }
}

hipError_t launch_batch_items(int prec, const BatchArgs &b, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (prec) {
  case G6MI_PREC_FP32: launch_batch_prec<G6MI_PREC_FP32>(b, grid, s); break;
  case G6MI_PREC_DS: launch_batch_prec<G6MI_PREC_DS>(b, grid, s); break;
  default: launch_batch_prec<G6MI_PREC_FP64>(b, grid, s);
  }
  return hipGetLastError();
}

hipError_t launch_batch_force(int prec, const BatchArgs &b, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  const hipError_t e = launch_batch_items(prec, b, grid, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(reduce_grid(grid)), dim3(kWG), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_nb_exact(int prec, const BatchArgs &b, int novf, hipStream_t s) {
  if (novf <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>(novf < 1024 ? novf : 1024));
  switch (prec) {
  case G6MI_PREC_FP32: hipLaunchKernelGGL(batch_nb_exact_kernel<G6MI_PREC_FP32>, grid, dim3(kWG), 0, s, b); break;
  case G6MI_PREC_DS: hipLaunchKernelGGL(batch_nb_exact_kernel<G6MI_PREC_DS>, grid, dim3(kWG), 0, s, b); break;
  default: hipLaunchKernelGGL(batch_nb_exact_kernel<G6MI_PREC_FP64>, grid, dim3(kWG), 0, s, b);
  }
  return hipGetLastError();
}

} // namespace g6mi
