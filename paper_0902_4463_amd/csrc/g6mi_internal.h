// Internal interface between the host-side state machine (g6mi_api.cpp) and
// the gfx950 kernels (g6mi_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/g6mi.h"

#include <cstddef>
#include <cstdint>

namespace g6mi {

// Build-time tuning knobs (defaults chosen by measurement on MI355X).
#ifndef G6MI_TILE
#define G6MI_TILE 256 // j-records staged in LDS per tile
#endif
#ifndef G6MI_GROUP
#define G6MI_GROUP 16 // j-records per nearest-neighbour group
#endif
#ifndef G6MI_SPATIAL_GROUP
#define G6MI_SPATIAL_GROUP 32 // j-records per group in the spatially ordered kernel
#endif
#ifndef G6MI_GROUP_UNROLL
#define G6MI_GROUP_UNROLL 1 // groups per unrolled loop body
#endif
#ifndef G6MI_FAR_K
#define G6MI_FAR_K 0.75f // far tile: gap to the i-box at least this many tile radii
#endif
#ifndef G6MI_FUSED_DEPTH
#define G6MI_FUSED_DEPTH 3 // records per lane in flight in the one-particle fused kernel
#endif
#ifndef G6MI_SELF_INF
#define G6MI_SELF_INF 1 // float32 self pair excluded through r^2 = +inf (one select)
#endif
#ifndef G6MI_NARROW_FOLD
#define G6MI_NARROW_FOLD 0 // narrow blocks: every group sum straight into float64
#endif
#ifndef G6MI_RSQ64_STEPS
#define G6MI_RSQ64_STEPS 1 // Newton-Raphson steps after the float64 1/sqrt estimate
#endif
#ifndef G6MI_WIDE_WAVES
#define G6MI_WIDE_WAVES 3 // register budget of the wide kernel: waves per SIMD (0: free)
#endif

constexpr int kWG = 256;          // lanes per workgroup: four wave64
constexpr int kTile = G6MI_TILE;  // j-records staged in LDS per tile
constexpr int kNbMax = 256;       // neighbour slots per i-particle
constexpr int kFusedDepth = G6MI_FUSED_DEPTH;
// Reduction of blocks of at most kFewMaxNi i-particles over more than 64
// splits: one workgroup per i-particle, at most kFewSplitsPerLane splits per lane.
#ifndef G6MI_FEW_MAX_NI
#define G6MI_FEW_MAX_NI 256
#endif
constexpr int kFewMaxNi = G6MI_FEW_MAX_NI;
constexpr int kFewSplitsPerLane = 4;

// Status words of one calculation in device memory (zeroed by the predictor
// launch): flags (bit 0 non-finite output, bit 1 neighbour overflow) and the
// number of i-particles queued for the exact overflow pass.
constexpr int kStatusFlags = 0;
constexpr int kStatusOverflowCount = 1;
constexpr int kStatusWords = 2;

// Predicted j-record sizes in bytes, one record per j-slot:
//   DS   : float4{x_hi, m}, float4{x_lo, 0}, float4{v, 0}  = 48 B
//   FP32 : float4{x, m},    float4{v, 0}                    = 32 B
//   FP64 : double4{x, m},   double4{v, 0}                   = 64 B
size_t pred_record_bytes(int prec);

// j-memory master copy on the device: float64 structure of arrays with
// `cap` slots; x, v, a2, j6 are [3][cap] (component-major) for coalesced
// predictor loads.
struct JMem {
  double *t = nullptr, *m = nullptr;
  double *x = nullptr, *v = nullptr, *a2 = nullptr, *j6 = nullptr;
  int *index = nullptr;
  size_t cap = 0;
};

struct ForceArgs {
  const void *jpred = nullptr; // predicted j-records, nj of them
  int nj = 0;
  int ni = 0;
  const double *xi = nullptr;  // [ni][3]
  const double *vi = nullptr;  // [ni][3]
  const double *h2 = nullptr;  // [ni]
  const int *islot = nullptr;  // [ni], own j-slot or -1
  double eps2 = 0.0;
  int ipw = kWG;               // i-particles per workgroup, power of two
  int log2ipw = 8;
  // outputs of the j-split s in [0, nsplit), component-major:
  double *part = nullptr;      // [nsplit][7][ni]: acc xyz, jerk xyz, sum m/r
  double *nn_r2 = nullptr;     // [nsplit][ni]
  int *nn_slot = nullptr;      // [nsplit][ni]
  int *nb_count = nullptr;     // [ni]   (zeroed by the predictor launch; see force_fused)
  int *nb_slot = nullptr;      // [ni][kNbMax]
};

hipError_t launch_predict(int prec, int nj, double ti, const JMem &jm,
                          void *out, int *nb_count, int ni, int *status,
                          hipStream_t s);

hipError_t launch_force(int prec, bool nbl, const ForceArgs &a, int nsplit,
                        hipStream_t s);

// One i-block of at most kWG i-particles (a.ipw <= kWG) with the predictor
// fused into the tile load: reads the j-memory jm at time ti instead of
// a.jpred, counts neighbours in nb_work (all zero before the launch; the
// reduction with the same nb_work clears it again) and clears the status
// words itself.
hipError_t launch_force_fused(int prec, bool nbl, const ForceArgs &a, const JMem &jm, double ti,
                              int *nb_work, int *status, int nsplit, hipStream_t s);

// Device address and size of the calling thread's current device's static
// scratch array (g6mi_calc_device_noalloc); `device` must be current.  The
// address is looked up once per device and kept.
hipError_t scratch_region(int device, void **ptr, size_t *bytes);

// Clear n ints with a kernel (no memset node when captured in a graph).
hipError_t launch_zero(int n, int *p, hipStream_t s);

// iperm: row of the partials at each position (spatially ordered blocks),
// or null where partials sit at their own rows.  nb_work: the counters of a
// force_fused launch (moved to nb_count and cleared), or null.
hipError_t launch_reduce(int nsplit, int ni, const int *iperm, const double *part,
                         const double *nn_r2, const int *nn_slot,
                         const int *jindex, int *nb_count, int *nb_slot,
                         bool nbl, double *acc, double *jerk, double *pot,
                         int *nnb, double *r2nn, int *status, int *ovf_list,
                         hipStream_t s, int *nb_work = nullptr);

// Rebuild the lists of the novf overflowed i-particles queued by the
// reduction (see reduce_kernel) with the kNbMax smallest indices.
hipError_t launch_nb_exact(int prec, const ForceArgs &a, const int *jindex,
                           const int *status, const int *ovf_list, int novf,
                           hipStream_t s);

// The exact overflow pass after a force_fused launch (records predicted
// again from jm at ti).
hipError_t launch_nb_exact_fused(int prec, const ForceArgs &a, const JMem &jm, double ti,
                                 const int *status, const int *ovf_list, int novf, hipStream_t s);

// Scatter nd staged records into the j-memory.  rec is [nd][16] doubles:
// t, m, x[3], v[3], a2[3], j6[3], index (as double), pad; slots is [nd].
hipError_t launch_scatter(int nd, const int *slots, const double *rec,
                          const JMem &jm, hipStream_t s);

// Copy nj records given as device arrays (row-major [nj][3] vectors) into
// slots 0..nj-1 of the j-memory.
hipError_t launch_load(int nj, const double *t, const double *m,
                       const int *index, const double *x, const double *v,
                       const double *a2, const double *j6, const JMem &jm,
                       hipStream_t s);

// ------------------------------------------ spatially ordered DS blocks

// Device buffers of the spatial ordering (g6mi_spatial.hip).
struct SpatialBufs {
  unsigned *box = nullptr;                       // [6] j box as order keys
  unsigned *keys_in = nullptr, *keys_out = nullptr; // [max(nj, ni)]
  int *vals_in = nullptr;                        // [max(nj, ni)]
  int *jperm = nullptr;                          // [nj] slot at each sorted position
  int *iperm = nullptr;                          // [ni] i-row at each sorted position
  int *inv = nullptr;                            // [nj] sorted position of each slot
  float4 *sorted = nullptr;                      // [nj][3] DS records in sorted order
  float4 *tinfo = nullptr;                       // [ntiles][4] centre, radius, box
  double *sxi = nullptr, *svi = nullptr;         // [ni][3] i-state in sorted order
  double *sh2 = nullptr;                         // [ni]
  int *sislot = nullptr;                         // [ni]
  int *spos = nullptr;                           // [ni] sorted position of the i-particle's own record, or -1
  void *temp = nullptr;                          // radix-sort scratch
  size_t temp_bytes = 0;
};

struct SpatialArgs {
  const int *iperm = nullptr;
  const int *spos = nullptr;
  const float4 *tinfo = nullptr;
};

// Scratch bytes of a radix sort of n (key, index) pairs.
hipError_t spatial_sort_bytes(int n, size_t *bytes);
// Box, keys, sorts of j and i, sorted records, tile table and the i-state
// gathered into sorted order.
hipError_t launch_spatial_prep(const SpatialBufs &b, int nj, int ni, const void *jpred, const double *xi,
                               const double *vi, const double *h2, const int *islot, hipStream_t s);
// The DS interaction over b.sorted and the sorted i-state (a holds the
// unsorted arrays); i-blocks of 512; partials at sorted positions (reduce
// with iperm = b.iperm).
hipError_t launch_force_spatial(bool nbl, const ForceArgs &a, const SpatialBufs &b, int nsplit, hipStream_t s);

// ------------------------------------------ batched multi-cluster launch

// Smallest i-block the batch plan uses when it cuts a cluster's block into
// more i-blocks for occupancy; bounds the work items at
// (ni_total / kBatchMinIpw + clusters + 1) * max_split.
#ifndef G6MI_BATCH_MIN_IPW
#define G6MI_BATCH_MIN_IPW 32
#endif
constexpr int kBatchMinIpw = G6MI_BATCH_MIN_IPW;

// Waves per SIMD of the narrow-only batch kernel (one i-particle per lane;
// its registers fit four).
constexpr int kNarrowWaves = 4;

// Launch policy of a batch (see BatchPlan): item_work = work per item in
// units of 128 lane-pairs (a quarter of one tile x 512 i-particles), wide_min = smallest cluster block
// that uses two i-particles per lane, max_split = cap on j-splits per
// cluster (bounds the partial-sum buffer).
struct BatchTune {
  int item_work = 8;
  int wide_min = 512;
  int max_split = 64;
};

// Per-cluster plan written by the plan kernel: i-particles per workgroup
// (512 = two per lane), j-splits and tiles per split, i-blocks, the
// cluster's first i-block counter, first work item and first partial entry,
// and its block size (0 for a skipped cluster).
// Its work items are item0 .. item0 + nib * nsplit - 1, item item0 + r
// being i-block r / nsplit, j-split r % nsplit.
struct BatchPlan {
  int ipw, log2ipw, nsplit, per, nib, ib0, item0, ni;
  long long pbase;
};

// Workgroups of a batch reduction (batch_reduce_kernel, hs_correct_kernel)
// for a persistent grid of `grid`: kReduceGridMul times as many, so that
// the i-blocks of a small batch are cut into parts (reduce_parts) and
// their split sums run with more loads in flight.
#ifndef G6MI_REDUCE_GRID_MUL
#define G6MI_REDUCE_GRID_MUL 4
#endif
constexpr int kReduceGridMul = G6MI_REDUCE_GRID_MUL;
__host__ __device__ constexpr int reduce_grid(int grid) { return grid * kReduceGridMul; }

// Most workgroups with rows in hs_correct_kernel: each ends with one atomic
// on the next block time, and a burst of them on one address queues up.
#ifndef G6MI_HS_REDUCE_WGS
#define G6MI_HS_REDUCE_WGS 256
#endif
constexpr int kHsReduceWgs = G6MI_HS_REDUCE_WGS;

// Work-queue state (written by the plan kernel): one counter per XCD group
// of workgroups (see batch_kernel), the number of items and of i-blocks.
constexpr int kQueues = 8;
struct BatchWork {
  int head[kQueues];
  int nitems, nib;
};

struct BatchArgs {
  const g6mi_cluster *cl = nullptr; // [ncl] descriptors in device memory
  BatchPlan *plan = nullptr;        // [ncl]
  int *item_cl = nullptr;           // [item_cap] cluster of each work item
  BatchWork *work = nullptr;
  int ncl = 0, nj_set = 0, ni_total = 0, item_cap = 0;
  int grid = 1;            // persistent workgroups of batch_kernel
  int wide = 1;            // 0: no cluster can take wide blocks (tune.wide_min > ni_total), and the
                           // batch runs the narrow-only kernel, whose registers allow more waves
  BatchTune tune;
  JMem jm;
  ForceArgs fa;            // i-arrays over rows 0..ni_total-1; nb_count, nb_slot
  double *part = nullptr;  // [7][pcap] split partials
  double *nn_r2 = nullptr; // [pcap]
  int *nn_slot = nullptr;  // [pcap]
  size_t pcap = 0;
  int *ib_cl = nullptr;    // [ni_total] cluster of each i-block (at most one per row)
  int nbl = 1;
  double *acc = nullptr, *jerk = nullptr, *pot = nullptr, *r2nn = nullptr;
  int *nnb = nullptr, *status = nullptr, *ovf_list = nullptr, *ovf_tag = nullptr;
};

// Rows cleared per workgroup of the plan launch besides workgroup 0.
constexpr int kPlanZeroChunk = 4096;

hipError_t launch_batch_plan(const BatchArgs &b, hipStream_t s);
// the persistent kernel and the reduction
hipError_t launch_batch_force(int prec, const BatchArgs &b, int grid, hipStream_t s);
// the persistent kernel alone (its partials reduced by the caller's launch)
hipError_t launch_batch_items(int prec, const BatchArgs &b, int grid, hipStream_t s);
hipError_t launch_batch_nb_exact(int prec, const BatchArgs &b, int novf, hipStream_t s);

// Status flag of the batched launch: a cluster descriptor was out of range
// or non-finite and its cluster was skipped.
constexpr int kFlagBadCluster = 4;

// ------------------------------------------ device-resident block steps

// Control block of the device-resident Hermite integrator (device memory).
//
// Block times as order keys (the minimum over the grid is one atomicMin):
// key[phase] holds this step's block time t_b; key[phase ^ 1] gathers the
// next one, the minimum of t + dt over the particles the selection leaves
// alone and over the corrected ones.  The publish launch between the two
// clears key[phase] and flips phase.
struct HermiteCtl {
  unsigned long long key[2];
  int phase;
  int ni_count;                 // particles selected so far in this step
  int done;                     // 1: no particle is due at or before t_end
  int flags;                    // bit 0: a non-finite force
  long long block_steps, particle_steps;
  double t_end;                 // run limit, set by the host
  double time;                  // time of the last completed block step
  g6mi_cluster desc;            // the current block as a one-cluster batch
};

// The integrator state is the j-memory (slots 0..n-1: t, m, x, v, a/2,
// jerk/6, index) plus a and jerk themselves, the step and the potential.
struct HermiteArgs {
  HermiteCtl *ctl = nullptr;
  JMem jm;
  double *acc = nullptr, *jrk = nullptr;  // [3][cap] at each particle's own time
  double *dt = nullptr, *pot = nullptr;   // [cap]
  int n = 0;
  int *active = nullptr;                  // [n] slots of the block, in selection order
  double *xi = nullptr, *vi = nullptr;    // [n][3] block predicted to the block time
  double *h2i = nullptr;                  // [n]
  double *acc1 = nullptr, *jrk1 = nullptr, *pot1 = nullptr; // [n][3], [n][3], [n] new forces
  double eps2 = 0, h2 = 0, eta = 0, eta_s = 0, dt_max = 0, dt_min = 0;
};

hipError_t launch_hs_reset(const HermiteArgs &h, hipStream_t s);
// the block due at the next block time, its descriptor and its one-cluster
// batch plan in b (two launches)
hipError_t launch_hs_select(const HermiteArgs &h, const BatchArgs &b, hipStream_t s);
// after the first force evaluation (a whole batched force launch): store a,
// jerk and potential and pick the first steps
hipError_t launch_hs_start(const HermiteArgs &h, hipStream_t s);
// after launch_batch_items: the batch reduction, corrector and new steps in
// one launch of `grid` workgroups
hipError_t launch_hs_correct(const HermiteArgs &h, const BatchArgs &b, int grid, hipStream_t s);

} // namespace g6mi
