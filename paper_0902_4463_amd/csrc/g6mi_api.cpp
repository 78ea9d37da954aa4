// Host side of libg6mi: handle state, j-memory staging, launch-shape choice
// and the exported C ABI declared in include/g6mi.h.
//
// One calculation enqueues, in order on one HIP stream:
//   [H2D of staged j-records + scatter kernel]   (only slots changed since
//                                                  the last calculation)
//   [H2D of the i-block]                          (host path only)
//   predict_kernel -> force_kernel -> reduce_kernel
//   [D2H of the results]                          (host path only)
// which is the CPU/GPU split of Sec. 2.1: the j-particles are predicted on
// the GPU, and only corrected particles and the i-block cross the bus.

#include "g6mi_internal.h"
#include "../../include/g6mi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#define G6MI_API extern "C" __attribute__((visibility("default")))

namespace {

using namespace g6mi;

constexpr int kRecDoubles = 16; // staged j-record: t m x3 v3 a2(3) j6(3) index pad

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct PinBuf {
  void *p = nullptr;
  size_t bytes = 0;
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
};

size_t round_up(size_t n, size_t q) { return (n + q - 1) / q * q; }

hipError_t ensure(DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return hipSuccess;
  b.release();
  const size_t nb = round_up(std::max<size_t>(bytes, 256), size_t(1) << 16);
  hipError_t e = hipMalloc(&b.p, nb);
  if (e == hipSuccess) b.bytes = nb;
  else b.p = nullptr;
  return e;
}

hipError_t ensure(PinBuf &b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return hipSuccess;
  b.release();
  const size_t nb = round_up(std::max<size_t>(bytes, 256), size_t(1) << 16);
  hipError_t e = hipHostMalloc(&b.p, nb, hipHostMallocDefault);
  if (e == hipSuccess) b.bytes = nb;
  else b.p = nullptr;
  return e;
}

struct Handle {
  bool open = false;
  int device = 0;
  hipStream_t stream = nullptr;
  int ncu = 0, clock_mhz = 0;
  std::string arch;
  int prec = G6MI_PREC_DS;
  bool nbl = true;
  int spatial = 1; // 0 off, 1 for large DS blocks, 2 always (DS)
  bool fuse = true; // one-block calls predict their tiles in the interaction kernel
  int user_ipw = 0, user_nsplit = 0;
  int shape[4] = {0, 0, 0, 0};
  std::string err;

  // host master copy of the j-memory, kRecDoubles per slot
  std::vector<double> h_rec;
  std::vector<int> h_index;
  std::vector<unsigned char> h_set, h_dirty;
  std::vector<int> dirty;
  size_t n_contig = 0; // slots 0..n_contig-1 have all been set
  std::unordered_map<int, int> slot_of;
  double ti = 0.0;

  // device j-memory
  JMem jm;
  DevBuf d_jm, d_pred, d_stage;
  PinBuf h_stage;
  hipEvent_t stage_ev = nullptr;
  bool stage_busy = false;

  // host-path i-block and outputs
  DevBuf d_i, d_out;
  PinBuf h_i, h_out;

  // work buffers
  DevBuf d_part, d_nnr2, d_nnslot, d_nbcount, d_nblist, d_flags, d_ovf;
  // neighbour counters of the fused path: all zero between calculations
  // (each reduction clears the rows it used); nbwork_ok is false until a
  // new buffer has been cleared or after a calculation that did not reach
  // its reduction
  DevBuf d_nbwork;
  bool nbwork_ok = false;
  DevBuf d_sp; // spatial ordering: one allocation cut into SpatialBufs
  SpatialBufs sp;

  // calculation state
  bool pending = false;
  int pending_err = 0;
  int c_nj = 0, c_ni = 0;
  double c_eps2 = 0.0;
  std::vector<int> c_index;
  hipStream_t c_stream = nullptr;
  ForceArgs c_args;        // interaction arguments of the last calculation
  bool c_fused = false;    // ... made by force_fused (no predicted records kept)
  double c_ti = 0.0;
  int *c_flags = nullptr, *c_ovf = nullptr; // its status words and overflow queue
  int c_prec = G6MI_PREC_DS;
  bool c_nbl = true;
  bool c_have = false;     // a calculation was enqueued and not superseded
  bool res_valid = false;  // host results of the last host-path calc
  std::vector<int> r_nnb;
  std::vector<double> r_r2nn;
  bool nb_read = false;
  bool nb_exact_done = false; // overflow pass run for the last calculation
  std::vector<int> r_nbcount, r_nblist;

  // timing: one set of four events per timed calculation since the last
  // g6mi_enable_timing / g6mi_timing_totals, at most kTimingRing sets
  bool timing = false;
  int n_timed = 0;
  std::vector<std::array<hipEvent_t, 4>> evs;

  // batched calculations
  BatchTune btune;
  int b_wg_per_cu = 0; // 0: as many as the kernel's occupancy allows
  DevBuf d_cl, d_plan, d_items, d_bwork, d_ibcl;
  PinBuf h_cl;
  hipEvent_t cl_ev = nullptr;
  bool cl_busy = false;
  bool use_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  bool c_batch = false;    // the last calculation was a batch
  BatchArgs c_bargs;

  // device-resident block steps
  struct {
    bool ready = false;
    int n = 0;
    HermiteArgs a;
    double *jm_t = nullptr; // the j-memory the state lives in
    size_t cap = 0;
    DevBuf d_ctl, d_state, d_block;
    PinBuf h_ctl;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
  } hs;
};

constexpr int kTimingRing = 4096;

Handle g_h[G6MI_MAX_HANDLES];
std::mutex g_mu;
std::string g_err;

int fail(Handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  else g_err = msg;
  return code;
}

int hip_fail(Handle *h, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(h, e == hipErrorOutOfMemory ? G6MI_ENOMEM : G6MI_EDEVICE, m);
}

#define HIPCHK(h, call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call);                     \
  } while (0)

Handle *get_open(int id) {
  if (id < 0 || id >= G6MI_MAX_HANDLES) {
    g_err = "invalid handle id";
    return nullptr;
  }
  Handle *h = &g_h[id];
  if (!h->open) {
    h->err = "handle not open";
    return nullptr;
  }
  return h;
}

int code_for_missing(int id) {
  return (id < 0 || id >= G6MI_MAX_HANDLES) ? G6MI_EINVAL : G6MI_ESTATE;
}

int parse_precision(const char *s, int dflt) {
  if (!s) return dflt;
  std::string v(s);
  std::transform(v.begin(), v.end(), v.begin(), ::tolower);
  if (v == "fp32" || v == "sp") return G6MI_PREC_FP32;
  if (v == "ds") return G6MI_PREC_DS;
  if (v == "fp64" || v == "dp") return G6MI_PREC_FP64;
  return dflt;
}

void grow_host(Handle &h, size_t need) {
  if (h.h_index.size() >= need) return;
  size_t n = std::max<size_t>(1024, h.h_index.size());
  while (n < need) n *= 2;
  h.h_rec.resize(n * kRecDoubles, 0.0);
  h.h_index.resize(n, -1);
  h.h_set.resize(n, 0);
  h.h_dirty.resize(n, 0);
}

void mark_dirty(Handle &h, int slot) {
  if (!h.h_dirty[slot]) {
    h.h_dirty[slot] = 1;
    h.dirty.push_back(slot);
  }
}

// Device j-memory with room for `need` slots.  A reallocation re-uploads
// every set slot from the host master copy.
int ensure_jmem(Handle &h, size_t need) {
  if (need <= h.jm.cap && h.jm.t) return 0;
  size_t cap = std::max<size_t>(4096, h.jm.cap);
  while (cap < need) cap *= 2;
  HIPCHK(&h, hipStreamSynchronize(h.stream));
  h.d_jm.release();
  h.jm = JMem{};
  const size_t bytes = cap * (14 * sizeof(double) + sizeof(int));
  HIPCHK(&h, ensure(h.d_jm, bytes));
  double *b = static_cast<double *>(h.d_jm.p);
  h.jm.t = b;
  h.jm.m = b + cap;
  h.jm.x = b + 2 * cap;
  h.jm.v = b + 5 * cap;
  h.jm.a2 = b + 8 * cap;
  h.jm.j6 = b + 11 * cap;
  h.jm.index = reinterpret_cast<int *>(b + 14 * cap);
  h.jm.cap = cap;
  HIPCHK(&h, hipMemsetAsync(h.d_jm.p, 0, bytes, h.stream));
  for (size_t k = 0; k < std::min(h.h_set.size(), cap); ++k)
    if (h.h_set[k]) mark_dirty(h, static_cast<int>(k));
  return 0;
}

// Upload the staged j-records on stream s: pack them into pinned memory, one
// H2D copy, then a scatter kernel into the structure-of-arrays master.
int upload_dirty(Handle &h, hipStream_t s) {
  if (h.dirty.empty()) return 0;
  const size_t nd = h.dirty.size();
  if (h.stage_busy) {
    HIPCHK(&h, hipEventSynchronize(h.stage_ev));
    h.stage_busy = false;
  }
  const size_t rec_bytes = nd * kRecDoubles * sizeof(double);
  const size_t bytes = rec_bytes + nd * sizeof(int);
  HIPCHK(&h, ensure(h.h_stage, bytes));
  HIPCHK(&h, ensure(h.d_stage, bytes));
  double *rec = static_cast<double *>(h.h_stage.p);
  int *slots = reinterpret_cast<int *>(static_cast<char *>(h.h_stage.p) + rec_bytes);
  for (size_t q = 0; q < nd; ++q) {
    const int k = h.dirty[q];
    std::memcpy(rec + q * kRecDoubles, &h.h_rec[static_cast<size_t>(k) * kRecDoubles],
                kRecDoubles * sizeof(double));
    slots[q] = k;
    h.h_dirty[k] = 0;
  }
  h.dirty.clear();
  HIPCHK(&h, hipMemcpyAsync(h.d_stage.p, h.h_stage.p, bytes, hipMemcpyHostToDevice, s));
  const double *drec = static_cast<const double *>(h.d_stage.p);
  const int *dslots = reinterpret_cast<const int *>(static_cast<char *>(h.d_stage.p) + rec_bytes);
  HIPCHK(&h, launch_scatter(static_cast<int>(nd), dslots, drec, h.jm, s));
  HIPCHK(&h, hipEventRecord(h.stage_ev, s));
  h.stage_busy = true;
  return 0;
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Launch shape.  i-particles per workgroup: 512 (two per lane) for blocks
// of at least 512, else the smallest power of two covering the block, at
// most 256 (one per lane); below 256 the spare lanes split the j-tile among
// themselves (Sec. 2.3, Fig. accMP1).
// j-splits: enough workgroups for G6MI_WG_PER_CU per compute unit (Sec. 2.3,
// Fig. accGPU splits j over all multiprocessors), each split at least
// kMinTiles tiles long.  Many short workgroups keep the last round on each
// CU small (measured: 8 splits of 2^20 j beat 1 split by 7%).
#ifndef G6MI_WG_PER_CU
#define G6MI_WG_PER_CU 64
#endif
constexpr int kWaveTarget = G6MI_WG_PER_CU;
constexpr int kMinTiles = 8;
constexpr int kOneSplits = 256;

// Spatial ordering (g6mi_spatial.hip) for double-single blocks of at least
// this many i-particles against at least two tiles (automatic mode).  The
// ordering costs two sorts per call (about 0.5 ms at 2^20 j-particles) and
// pays only when the active particles are dense enough for a workgroup's 512
// of them to fill a compact box: measured against 2^20 Plummer j-particles,
// random active blocks of 2^12 .. 2^14 ran slower ordered, 2^16 and up
// faster (8% at 2^16, 17% at 2^20).
constexpr int kSpatialMinNi = 65536;

bool use_spatial(const Handle &h, int ni, int nj) {
  if (h.prec != G6MI_PREC_DS || ni <= 0 || nj <= 0) return false;
  if (h.spatial == 2) return true;
  return h.spatial == 1 && !h.user_ipw && ni >= kSpatialMinNi && nj >= 2 * kTile;
}

// The predictor fused into the interaction (force_fused) for a call whose
// block is one narrow i-block: every j-tile is then predicted once either
// way, and the predicted records need not go through HBM.
bool use_fused(const Handle &h, bool spatial, int ipw, int ni, int nj) {
  return h.fuse && !spatial && ni > 0 && nj > 0 && ipw <= kWG && ni <= ipw;
}

void choose_shape(Handle &h, int ni, int nj, int &ipw, int &nsplit, bool may_order = true) {
  const int ntiles = (nj + kTile - 1) / kTile;
  if (may_order && use_spatial(h, ni, nj)) ipw = 2 * kWG;
  else if (h.user_ipw) ipw = h.user_ipw;
  else if (ni >= 2 * kWG) ipw = 2 * kWG; // two i-particles per lane
  else {
    ipw = kWG;
    while (ipw > 1 && ipw / 2 >= ni) ipw /= 2;
  }
  const long nib = (ni + ipw - 1) / ipw;
  if (h.user_nsplit) {
    nsplit = std::max(1, std::min(h.user_nsplit, std::max(1, ntiles)));
  } else {
    // enough workgroups that the last round on each compute unit is a small
    // fraction of the work, each split at least kMinTiles tiles long
    const long target = static_cast<long>(kWaveTarget) * std::max(1, h.ncu);
    nsplit = static_cast<int>(std::max(1L, (target + nib - 1) / std::max(1L, nib)));
    nsplit = std::max(1, std::min(nsplit, std::max(1, ntiles / kMinTiles)));
    // one particle with the predictor fused in: the interaction streams the
    // j-memory whatever the split count, and the reduction of 256 splits
    // takes one round of loads where 512 take two (measured at 2^20 j:
    // 25.3-26.3 against 26.4-27.1 us per call)
    if (ipw == 1 && h.fuse) nsplit = std::min(nsplit, kOneSplits);
  }
  nsplit = std::min(nsplit, 4096);
}

// Buffers of the spatial ordering for nj records and ni i-particles.
int ensure_spatial(Handle &h, int nj, int ni) {
  const size_t n = static_cast<size_t>(std::max(nj, ni)), j = static_cast<size_t>(nj), i = static_cast<size_t>(ni);
  const size_t ntiles = (j + kTile - 1) / kTile;
  size_t temp = 0;
  HIPCHK(&h, spatial_sort_bytes(static_cast<int>(n), &temp));
  auto al = [](size_t b) { return round_up(std::max<size_t>(b, 1), 256); };
  const size_t sizes[] = {al(6 * sizeof(unsigned)), al(n * 4), al(n * 4), al(n * 4), al(j * 4), al(i * 4),
                          al(j * 4), al(j * 48), al(ntiles * 64), al(i * 24), al(i * 24), al(i * 8), al(i * 4),
                          al(i * 4), al(temp)};
  constexpr int kParts = sizeof(sizes) / sizeof(sizes[0]);
  size_t total = 0;
  for (size_t b : sizes) total += b;
  HIPCHK(&h, ensure(h.d_sp, total));
  char *p = static_cast<char *>(h.d_sp.p);
  void *parts[kParts];
  for (int k = 0; k < kParts; ++k) {
    parts[k] = p;
    p += sizes[k];
  }
  SpatialBufs &b = h.sp;
  b.box = static_cast<unsigned *>(parts[0]);
  b.keys_in = static_cast<unsigned *>(parts[1]);
  b.keys_out = static_cast<unsigned *>(parts[2]);
  b.vals_in = static_cast<int *>(parts[3]);
  b.jperm = static_cast<int *>(parts[4]);
  b.iperm = static_cast<int *>(parts[5]);
  b.inv = static_cast<int *>(parts[6]);
  b.sorted = static_cast<float4 *>(parts[7]);
  b.tinfo = static_cast<float4 *>(parts[8]);
  b.sxi = static_cast<double *>(parts[9]);
  b.svi = static_cast<double *>(parts[10]);
  b.sh2 = static_cast<double *>(parts[11]);
  b.sislot = static_cast<int *>(parts[12]);
  b.spos = static_cast<int *>(parts[13]);
  b.temp = parts[14];
  b.temp_bytes = sizes[14];
  return 0;
}

// Work buffers of one single-system calculation.
struct CalcBufs {
  void *pred = nullptr;                    // predicted j-records (not with the fused kernel)
  double *part = nullptr, *nnr2 = nullptr; // split partials
  int *nnslot = nullptr;
  int *nbcount = nullptr, *nblist = nullptr;
  int *flags = nullptr, *ovf = nullptr;    // status words, overflow queue
  int *nbwork = nullptr;                   // fused kernel's neighbour counters
  int nbwork_n = 0;                        // ... their number
  bool nbwork_zero = false;                // nbwork is known to be all zero
};

// Bytes of the work buffers of a calculation of shape (ipw, nsplit) over
// nj j-slots and ni i-particles, in the order and alignment of carve_bufs.
size_t calc_bytes(int prec, bool fused, int nj, int ni, int nsplit) {
  const size_t n = static_cast<size_t>(std::max(ni, 1)), ns = static_cast<size_t>(nsplit);
  size_t b = 0;
  auto add = [&](size_t x) { b += round_up(x, 256); };
  add(fused ? 0 : std::max<size_t>(1, nj) * pred_record_bytes(prec));
  add(ns * 7 * n * sizeof(double));
  add(ns * n * sizeof(double));
  add(ns * n * sizeof(int));
  add(n * sizeof(int));
  add(n * kNbMax * sizeof(int));
  add(64);
  add(2 * n * sizeof(int));
  add(fused ? n * sizeof(int) : 0);
  return b;
}

// The same buffers cut from one region of at least calc_bytes bytes.
CalcBufs carve_bufs(void *base, int prec, bool fused, int nj, int ni, int nsplit) {
  const size_t n = static_cast<size_t>(std::max(ni, 1)), ns = static_cast<size_t>(nsplit);
  char *p = static_cast<char *>(base);
  auto take = [&](size_t x) {
    char *q = p;
    p += round_up(x, 256);
    return static_cast<void *>(q);
  };
  CalcBufs c;
  c.pred = take(fused ? 0 : std::max<size_t>(1, nj) * pred_record_bytes(prec));
  c.part = static_cast<double *>(take(ns * 7 * n * sizeof(double)));
  c.nnr2 = static_cast<double *>(take(ns * n * sizeof(double)));
  c.nnslot = static_cast<int *>(take(ns * n * sizeof(int)));
  c.nbcount = static_cast<int *>(take(n * sizeof(int)));
  c.nblist = static_cast<int *>(take(n * kNbMax * sizeof(int)));
  c.flags = static_cast<int *>(take(64));
  c.ovf = static_cast<int *>(take(2 * n * sizeof(int)));
  c.nbwork = fused ? static_cast<int *>(take(n * sizeof(int))) : nullptr;
  c.nbwork_n = fused ? static_cast<int>(n) : 0;
  if (fused) c.pred = nullptr;
  return c;
}

// The handle's own work buffers, grown as needed.
int handle_bufs(Handle &h, bool fused, int nj, int ni, int nsplit, CalcBufs &c) {
  const size_t n = static_cast<size_t>(std::max(ni, 1));
  if (!fused) HIPCHK(&h, ensure(h.d_pred, std::max<size_t>(1, nj) * pred_record_bytes(h.prec)));
  HIPCHK(&h, ensure(h.d_part, static_cast<size_t>(nsplit) * 7 * n * sizeof(double)));
  HIPCHK(&h, ensure(h.d_nnr2, static_cast<size_t>(nsplit) * n * sizeof(double)));
  HIPCHK(&h, ensure(h.d_nnslot, static_cast<size_t>(nsplit) * n * sizeof(int)));
  HIPCHK(&h, ensure(h.d_nbcount, n * sizeof(int)));
  HIPCHK(&h, ensure(h.d_nblist, n * kNbMax * sizeof(int)));
  HIPCHK(&h, ensure(h.d_flags, 64));
  HIPCHK(&h, ensure(h.d_ovf, 2 * n * sizeof(int)));
  c.pred = fused ? nullptr : h.d_pred.p;
  c.part = static_cast<double *>(h.d_part.p);
  c.nnr2 = static_cast<double *>(h.d_nnr2.p);
  c.nnslot = static_cast<int *>(h.d_nnslot.p);
  c.nbcount = static_cast<int *>(h.d_nbcount.p);
  c.nblist = static_cast<int *>(h.d_nblist.p);
  c.flags = static_cast<int *>(h.d_flags.p);
  c.ovf = static_cast<int *>(h.d_ovf.p);
  if (fused) {
    const size_t before = h.d_nbwork.bytes;
    HIPCHK(&h, ensure(h.d_nbwork, n * sizeof(int)));
    if (h.d_nbwork.bytes != before) h.nbwork_ok = false;
    c.nbwork = static_cast<int *>(h.d_nbwork.p);
    c.nbwork_n = static_cast<int>(h.d_nbwork.bytes / sizeof(int));
    c.nbwork_zero = h.nbwork_ok;
  }
  return 0;
}

// Enqueue one calculation on stream s.  scratch == nullptr: the handle's own
// buffers (allocated as needed), the spatial ordering where it applies, and
// the timing events.  Otherwise every work buffer is cut from `scratch`
// (scratch_bytes long) and nothing is allocated: the calculation is not
// spatially ordered and not timed, and j-split counts are lowered until the
// buffers fit (G6MI_EINVAL when even one split does not).
int enqueue_calc(Handle &h, int nj, int ni, const int *d_islot, const double *d_xi,
                 const double *d_vi, const double *d_h2, double eps2, double *d_acc,
                 double *d_jerk, double *d_pot, int *d_nnb, double *d_r2nn, hipStream_t s,
                 void *scratch = nullptr, size_t scratch_bytes = 0) {
  const bool noalloc = scratch != nullptr;
  if (noalloc && !h.dirty.empty())
    return fail(&h, G6MI_ESTATE, "j-particles set on the host wait for an upload, which needs staging memory");
  if (!noalloc) {
    int rc = upload_dirty(h, s);
    if (rc) return rc;
  }
  int ipw, nsplit;
  choose_shape(h, ni, nj, ipw, nsplit, !noalloc);
  const bool spatial = !noalloc && use_spatial(h, ni, nj);
  // one i-block of at most kWG: the interaction kernel predicts its tiles
  const bool fused = use_fused(h, spatial, ipw, ni, nj);
  CalcBufs c;
  if (noalloc) {
    while (nsplit > 1 && calc_bytes(h.prec, fused, nj, ni, nsplit) > scratch_bytes) nsplit = (nsplit + 1) / 2;
    if (calc_bytes(h.prec, fused, nj, ni, nsplit) > scratch_bytes)
      return fail(&h, G6MI_EINVAL, "calculation too large for the static scratch buffer (nj or ni too large)");
    c = carve_bufs(scratch, h.prec, fused, nj, ni, nsplit);
  } else {
    int rc = handle_bufs(h, fused, nj, ni, nsplit, c);
    if (rc) return rc;
  }
  int *status = c.flags; // cleared by the predictor launch, or by force_fused

  h.shape[0] = ipw;
  h.shape[1] = nsplit;
  h.shape[2] = kTile;
  h.shape[3] = ((ni + ipw - 1) / ipw) * nsplit;
  hipEvent_t *ev = nullptr;
  if (!noalloc && h.timing && h.n_timed < kTimingRing) {
    if (static_cast<size_t>(h.n_timed) == h.evs.size()) {
      std::array<hipEvent_t, 4> q{};
      for (auto &e : q) HIPCHK(&h, hipEventCreate(&e));
      h.evs.push_back(q);
    }
    ev = h.evs[h.n_timed].data();
  }
  if (spatial) {
    int rc2 = ensure_spatial(h, nj, ni);
    if (rc2) return rc2;
  }
  if (fused) {
    if (!c.nbwork_zero) HIPCHK(&h, launch_zero(c.nbwork_n, c.nbwork, s));
    if (!noalloc) h.nbwork_ok = false; // until the reduction is enqueued
  }
  if (ev) HIPCHK(&h, hipEventRecord(ev[0], s));
  if (!fused) HIPCHK(&h, launch_predict(h.prec, nj, h.ti, h.jm, c.pred, c.nbcount, ni, status, s));
  if (spatial) HIPCHK(&h, launch_spatial_prep(h.sp, nj, ni, c.pred, d_xi, d_vi, d_h2, d_islot, s));
  if (ev) HIPCHK(&h, hipEventRecord(ev[1], s));
  ForceArgs a;
  a.jpred = c.pred;
  a.nj = nj;
  a.ni = ni;
  a.xi = d_xi;
  a.vi = d_vi;
  a.h2 = d_h2;
  a.islot = d_islot;
  a.eps2 = eps2;
  a.ipw = ipw;
  a.log2ipw = ilog2(ipw);
  a.part = c.part;
  a.nn_r2 = c.nnr2;
  a.nn_slot = c.nnslot;
  a.nb_count = c.nbcount;
  a.nb_slot = c.nblist;
  if (spatial) {
    HIPCHK(&h, launch_force_spatial(h.nbl, a, h.sp, nsplit, s));
  } else if (fused) {
    HIPCHK(&h, launch_force_fused(h.prec, h.nbl, a, h.jm, h.ti, c.nbwork, status, nsplit, s));
  } else {
    HIPCHK(&h, launch_force(h.prec, h.nbl, a, nsplit, s));
  }
  if (ev) HIPCHK(&h, hipEventRecord(ev[2], s));
  HIPCHK(&h, launch_reduce(nsplit, ni, spatial ? h.sp.iperm : nullptr, a.part, a.nn_r2, a.nn_slot, h.jm.index,
                           a.nb_count, a.nb_slot, h.nbl, d_acc, d_jerk, d_pot, d_nnb, d_r2nn, status, c.ovf, s,
                           c.nbwork));
  // the reduction clears the fused counters again (without lists nothing was counted)
  if (fused && !noalloc) h.nbwork_ok = true;
  if (ev) {
    HIPCHK(&h, hipEventRecord(ev[3], s));
    ++h.n_timed;
  }
  h.c_nj = nj;
  h.c_ni = ni;
  h.c_eps2 = eps2;
  h.c_stream = s;
  h.c_args = a;
  h.c_fused = fused;
  h.c_ti = h.ti;
  h.c_flags = status;
  h.c_ovf = c.ovf;
  h.c_prec = h.prec;
  h.c_nbl = h.nbl;
  h.c_have = true;
  h.c_batch = false;
  h.nb_read = false;
  h.nb_exact_done = false;
  return 0;
}

bool finite3(const double *p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

// Layout of the host-path i-block and result buffers (same on both sides).
struct IBlockLayout {
  size_t xi, vi, h2, islot, bytes;
  explicit IBlockLayout(size_t n) {
    xi = 0;
    vi = xi + 3 * n * sizeof(double);
    h2 = vi + 3 * n * sizeof(double);
    islot = h2 + n * sizeof(double);
    bytes = islot + n * sizeof(int);
  }
};
struct OutLayout {
  size_t acc, jerk, pot, r2nn, nnb, flags, bytes;
  explicit OutLayout(size_t n) {
    acc = 0;
    jerk = acc + 3 * n * sizeof(double);
    pot = jerk + 3 * n * sizeof(double);
    r2nn = pot + n * sizeof(double);
    nnb = r2nn + n * sizeof(double);
    flags = round_up(nnb + n * sizeof(int), 16);
    bytes = flags + 16;
  }
};

int firsthalf_impl(Handle &h, int nj, int ni, const int *index, const double (*xi)[3],
                   const double (*vi)[3], double eps2, const double *h2) {
  if (nj < 0 || static_cast<size_t>(nj) > h.n_contig)
    return fail(&h, G6MI_EINVAL, "nj exceeds the number of j-slots set from slot 0");
  if (ni < 0 || ni > G6MI_NI_MAX) return fail(&h, G6MI_EINVAL, "ni out of range");
  if (ni > 0 && (!index || !xi || !vi)) return fail(&h, G6MI_EINVAL, "null i-particle array");
  if (!std::isfinite(eps2) || eps2 < 0.0) return fail(&h, G6MI_EINVAL, "eps2 must be finite and >= 0");
  for (int i = 0; i < ni; ++i)
    if (!finite3(xi[i]) || !finite3(vi[i]) || (h2 && std::isnan(h2[i])))
      return fail(&h, G6MI_EINVAL, "non-finite i-particle data");
  int rc = ensure_jmem(h, std::max<size_t>(1, static_cast<size_t>(nj)));
  if (rc) return rc;
  const size_t n = static_cast<size_t>(std::max(ni, 1));
  IBlockLayout il(n);
  OutLayout ol(n);
  if (h.stage_busy) { // the i-block shares nothing with the j staging, but
    HIPCHK(&h, hipEventSynchronize(h.stage_ev)); // keep one staging fence
    h.stage_busy = false;
  }
  HIPCHK(&h, ensure(h.h_i, il.bytes));
  HIPCHK(&h, ensure(h.d_i, il.bytes));
  HIPCHK(&h, ensure(h.h_out, ol.bytes));
  HIPCHK(&h, ensure(h.d_out, ol.bytes));
  char *hi = static_cast<char *>(h.h_i.p);
  double *pxi = reinterpret_cast<double *>(hi + il.xi);
  double *pvi = reinterpret_cast<double *>(hi + il.vi);
  double *ph2 = reinterpret_cast<double *>(hi + il.h2);
  int *pis = reinterpret_cast<int *>(hi + il.islot);
  for (int i = 0; i < ni; ++i) {
    for (int d = 0; d < 3; ++d) {
      pxi[3 * i + d] = xi[i][d];
      pvi[3 * i + d] = vi[i][d];
    }
    ph2[i] = h2 ? h2[i] : 0.0;
    auto it = h.slot_of.find(index[i]);
    pis[i] = (it != h.slot_of.end() && it->second < nj) ? it->second : -1;
  }
  hipStream_t s = h.stream;
  HIPCHK(&h, hipMemcpyAsync(h.d_i.p, h.h_i.p, il.bytes, hipMemcpyHostToDevice, s));
  char *di = static_cast<char *>(h.d_i.p);
  char *dout = static_cast<char *>(h.d_out.p);
  rc = enqueue_calc(h, nj, ni, reinterpret_cast<const int *>(di + il.islot),
                    reinterpret_cast<const double *>(di + il.xi),
                    reinterpret_cast<const double *>(di + il.vi),
                    reinterpret_cast<const double *>(di + il.h2), eps2,
                    reinterpret_cast<double *>(dout + ol.acc),
                    reinterpret_cast<double *>(dout + ol.jerk),
                    reinterpret_cast<double *>(dout + ol.pot),
                    reinterpret_cast<int *>(dout + ol.nnb),
                    reinterpret_cast<double *>(dout + ol.r2nn), s);
  if (rc) return rc;
  HIPCHK(&h, hipMemcpyAsync(dout + ol.flags, h.c_flags, sizeof(int), hipMemcpyDeviceToDevice, s));
  HIPCHK(&h, hipMemcpyAsync(h.h_out.p, h.d_out.p, ol.bytes, hipMemcpyDeviceToHost, s));
  h.c_index.assign(index, index + ni);
  return 0;
}

int lasthalf_impl(int id, int nj, int ni, const int *index, double eps2, double (*acc)[3],
                  double (*jerk)[3], double *pot, int *nnbindex) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!h->pending) return fail(h, G6MI_ESTATE, "g6calc_lasthalf without g6calc_firsthalf");
  h->pending = false;
  if (h->pending_err) {
    h->c_have = false;
    return h->pending_err;
  }
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (nj != h->c_nj || ni != h->c_ni || eps2 != h->c_eps2 ||
      (ni > 0 && (!index || std::memcmp(index, h->c_index.data(), sizeof(int) * ni) != 0)))
    return fail(h, G6MI_EINVAL, "lasthalf arguments differ from firsthalf");
  if (ni > 0 && (!acc || !jerk || !pot)) return fail(h, G6MI_EINVAL, "null output array");
  const size_t n = static_cast<size_t>(std::max(ni, 1));
  OutLayout ol(n);
  const char *ho = static_cast<const char *>(h->h_out.p);
  const double *pa = reinterpret_cast<const double *>(ho + ol.acc);
  const double *pj = reinterpret_cast<const double *>(ho + ol.jerk);
  const double *pp = reinterpret_cast<const double *>(ho + ol.pot);
  const double *pr = reinterpret_cast<const double *>(ho + ol.r2nn);
  const int *pn = reinterpret_cast<const int *>(ho + ol.nnb);
  const int flags = *reinterpret_cast<const int *>(ho + ol.flags);
  for (int i = 0; i < ni; ++i) {
    for (int d = 0; d < 3; ++d) {
      acc[i][d] = pa[3 * i + d];
      jerk[i][d] = pj[3 * i + d];
    }
    pot[i] = pp[i];
    if (nnbindex) nnbindex[i] = pn[i];
  }
  h->r_nnb.assign(pn, pn + ni);
  h->r_r2nn.assign(pr, pr + ni);
  h->res_valid = true;
  return (ni > 0 && (flags & 1)) ? G6MI_WARN : G6MI_OK;
}

// ------------------------------------------------------------ batched path

// Partial sums of a batch: at most this many bytes (7 sums, r^2 and slot per
// i-particle and j-split); the j-split cap is lowered to fit.
constexpr size_t kBatchPartialBudget = size_t(4) << 30;
constexpr size_t kPartialEntryBytes = 7 * sizeof(double) + sizeof(double) + sizeof(int);
constexpr int kBatchMaxClusters = 1 << 20;

// Persistent workgroups per CU that the batch kernel's registers allow: the
// narrow-only kernel (no cluster of the batch can take wide blocks) fits four.
int batch_waves(int prec, bool narrow) { return narrow ? kNarrowWaves : prec == G6MI_PREC_FP64 ? 2 : 3; }

// Whether a batch over ni_total rows runs the narrow-only kernel: a cluster
// takes wide blocks from wide_min i-particles on, and none has more than
// ni_total.
bool batch_narrow(const Handle &h, int ni_total) { return h.btune.wide_min > ni_total; }

int batch_grid(const Handle &h, int prec, bool narrow) {
  const int w = h.b_wg_per_cu > 0 ? h.b_wg_per_cu : batch_waves(prec, narrow);
  return std::max(1, h.ncu) * w;
}

void destroy_graph(Handle &h) {
  if (h.gexec) (void)hipGraphExecDestroy(h.gexec);
  if (h.graph) (void)hipGraphDestroy(h.graph);
  h.gexec = nullptr;
  h.graph = nullptr;
  h.gkey.clear();
}

std::vector<uint64_t> graph_key(const Handle &h, const BatchArgs &b, int grid, hipStream_t s) {
  auto u = [](const void *p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); };
  return {u(b.cl), u(b.plan), u(b.item_cl), u(b.work), static_cast<uint64_t>(b.ncl),
          static_cast<uint64_t>(b.nj_set), static_cast<uint64_t>(b.ni_total),
          static_cast<uint64_t>(b.item_cap), static_cast<uint64_t>(b.tune.item_work),
          static_cast<uint64_t>(b.tune.wide_min), static_cast<uint64_t>(b.tune.max_split),
          u(b.jm.t), static_cast<uint64_t>(b.jm.cap), u(b.fa.xi), u(b.fa.vi), u(b.fa.h2),
          u(b.fa.islot), u(b.fa.nb_count), u(b.fa.nb_slot), u(b.part), u(b.nn_r2), u(b.nn_slot),
          static_cast<uint64_t>(b.pcap), u(b.ib_cl), static_cast<uint64_t>(b.nbl), u(b.acc),
          u(b.jerk), u(b.pot), u(b.r2nn), u(b.nnb), u(b.status), u(b.ovf_list), u(b.ovf_tag),
          static_cast<uint64_t>(h.prec), static_cast<uint64_t>(grid), u(s)};
}

// Plan kernel + persistent kernel on stream s, either launched directly
// (with the event `mid`, if any, recorded between them) or through a
// captured graph that is replayed while every argument stays the same
// (`mid` then recorded before the graph).
int launch_batch_all(Handle &h, const BatchArgs &b, int grid, hipStream_t s, hipEvent_t mid) {
  if (!h.use_graph) {
    HIPCHK(&h, launch_batch_plan(b, s));
    if (mid) HIPCHK(&h, hipEventRecord(mid, s));
    HIPCHK(&h, launch_batch_force(h.prec, b, grid, s));
    return 0;
  }
  if (mid) HIPCHK(&h, hipEventRecord(mid, s));
  std::vector<uint64_t> key = graph_key(h, b, grid, s);
  if (h.gexec && key == h.gkey) {
    HIPCHK(&h, hipGraphLaunch(h.gexec, s));
    return 0;
  }
  destroy_graph(h);
  HIPCHK(&h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_batch_plan(b, s);
  if (e == hipSuccess) e = launch_batch_force(h.prec, b, grid, s);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &g);
  if (e == hipSuccess) e = ec;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(&h, e, "batch graph capture");
  }
  h.graph = g;
  e = hipGraphInstantiate(&h.gexec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    h.gexec = nullptr;
    destroy_graph(h);
    return hip_fail(&h, e, "hipGraphInstantiate");
  }
  h.gkey = std::move(key);
  HIPCHK(&h, hipGraphLaunch(h.gexec, s));
  return 0;
}

// Work buffers and arguments of a batch (no launch).  nj_set bounds the
// j-slots the descriptors may name.
int prepare_batch(Handle &h, int ncl, const g6mi_cluster *d_cl, int ni_total, int nj_set, const int *d_islot,
                  const double *d_xi, const double *d_vi, const double *d_h2, double *d_acc,
                  double *d_jerk, double *d_pot, int *d_nnb, double *d_r2nn, BatchArgs &b) {
  const size_t n = static_cast<size_t>(std::max(ni_total, 1));
  BatchTune tune = h.btune;
  const size_t fit = kBatchPartialBudget / (n * kPartialEntryBytes);
  tune.max_split = static_cast<int>(std::max<size_t>(1, std::min<size_t>(tune.max_split, fit)));
  const size_t item_cap =
      (n / kBatchMinIpw + static_cast<size_t>(ncl) + 1) * static_cast<size_t>(tune.max_split);
  if (item_cap > static_cast<size_t>(INT_MAX)) return fail(&h, G6MI_EINVAL, "batch too large");
  const size_t pcap = n * static_cast<size_t>(tune.max_split);
  HIPCHK(&h, ensure(h.d_plan, std::max(ncl, 1) * sizeof(BatchPlan)));
  HIPCHK(&h, ensure(h.d_items, item_cap * sizeof(int)));
  HIPCHK(&h, ensure(h.d_bwork, sizeof(BatchWork)));
  HIPCHK(&h, ensure(h.d_ibcl, n * sizeof(int)));
  HIPCHK(&h, ensure(h.d_part, 7 * pcap * sizeof(double)));
  HIPCHK(&h, ensure(h.d_nnr2, pcap * sizeof(double)));
  HIPCHK(&h, ensure(h.d_nnslot, pcap * sizeof(int)));
  HIPCHK(&h, ensure(h.d_nbcount, n * sizeof(int)));
  HIPCHK(&h, ensure(h.d_nblist, n * kNbMax * sizeof(int)));
  HIPCHK(&h, ensure(h.d_flags, 64));
  HIPCHK(&h, ensure(h.d_ovf, 2 * n * sizeof(int)));

  b = BatchArgs{};
  b.cl = d_cl;
  b.plan = static_cast<BatchPlan *>(h.d_plan.p);
  b.item_cl = static_cast<int *>(h.d_items.p);
  b.work = static_cast<BatchWork *>(h.d_bwork.p);
  b.ncl = ncl;
  b.nj_set = nj_set;
  b.ni_total = ni_total;
  b.item_cap = static_cast<int>(item_cap);
  b.wide = batch_narrow(h, ni_total) ? 0 : 1;
  b.grid = batch_grid(h, h.prec, b.wide == 0);
  b.tune = tune;
  b.jm = h.jm;
  b.fa.xi = d_xi;
  b.fa.vi = d_vi;
  b.fa.h2 = d_h2;
  b.fa.islot = d_islot;
  b.fa.ni = ni_total;
  b.fa.nb_count = static_cast<int *>(h.d_nbcount.p);
  b.fa.nb_slot = static_cast<int *>(h.d_nblist.p);
  b.part = static_cast<double *>(h.d_part.p);
  b.nn_r2 = static_cast<double *>(h.d_nnr2.p);
  b.nn_slot = static_cast<int *>(h.d_nnslot.p);
  b.pcap = pcap;
  b.ib_cl = static_cast<int *>(h.d_ibcl.p);
  b.nbl = h.nbl ? 1 : 0;
  b.acc = d_acc;
  b.jerk = d_jerk;
  b.pot = d_pot;
  b.nnb = d_nnb;
  b.r2nn = d_r2nn;
  b.status = static_cast<int *>(h.d_flags.p);
  b.ovf_list = static_cast<int *>(h.d_ovf.p);
  b.ovf_tag = b.ovf_list + n;
  return 0;
}

// Enqueue a batch whose ncl descriptors are at d_cl (device memory).
int enqueue_batch(Handle &h, int ncl, const g6mi_cluster *d_cl, int ni_total, const int *d_islot,
                  const double *d_xi, const double *d_vi, const double *d_h2, double *d_acc,
                  double *d_jerk, double *d_pot, int *d_nnb, double *d_r2nn, hipStream_t s) {
  int rc = ensure_jmem(h, std::max<size_t>(1, h.n_contig));
  if (rc) return rc;
  rc = upload_dirty(h, s);
  if (rc) return rc;
  BatchArgs b;
  rc = prepare_batch(h, ncl, d_cl, ni_total, static_cast<int>(h.n_contig), d_islot, d_xi, d_vi, d_h2, d_acc,
                     d_jerk, d_pot, d_nnb, d_r2nn, b);
  if (rc) return rc;
  const BatchTune &tune = b.tune;
  const int grid = b.grid;

  h.shape[0] = 0;
  h.shape[1] = tune.max_split;
  h.shape[2] = kTile;
  h.shape[3] = grid;
  hipEvent_t *ev = nullptr;
  if (h.timing && h.n_timed < kTimingRing) {
    if (static_cast<size_t>(h.n_timed) == h.evs.size()) {
      std::array<hipEvent_t, 4> q{};
      for (auto &e : q) HIPCHK(&h, hipEventCreate(&e));
      h.evs.push_back(q);
    }
    ev = h.evs[h.n_timed].data();
  }
  if (ev) HIPCHK(&h, hipEventRecord(ev[0], s));
  rc = launch_batch_all(h, b, grid, s, ev ? ev[1] : nullptr);
  if (rc) return rc;
  if (ev) {
    HIPCHK(&h, hipEventRecord(ev[2], s));
    HIPCHK(&h, hipEventRecord(ev[3], s));
    ++h.n_timed;
  }
  h.c_nj = 0;
  h.c_ni = ni_total;
  h.c_eps2 = 0.0;
  h.c_stream = s;
  h.c_prec = h.prec;
  h.c_nbl = h.nbl;
  h.c_have = true;
  h.c_batch = true;
  h.c_bargs = b;
  h.res_valid = false;
  h.nb_read = false;
  h.nb_exact_done = false;
  return 0;
}

int check_batch_args(Handle *h, int ncl, int ni_total, const int *d_islot, const double *d_xi,
                     const double *d_vi, const double *d_h2, const double *d_acc, const double *d_jerk,
                     const double *d_pot) {
  if (h->pending) return fail(h, G6MI_ESTATE, "a host-path calculation is pending");
  if (ncl < 0 || ncl > kBatchMaxClusters) return fail(h, G6MI_EINVAL, "ncl out of range");
  if (ni_total < 0 || ni_total > G6MI_NI_MAX) return fail(h, G6MI_EINVAL, "ni_total out of range");
  if (ni_total > 0 && (!d_islot || !d_xi || !d_vi || !d_h2 || !d_acc || !d_jerk || !d_pot))
    return fail(h, G6MI_EINVAL, "null device array");
  return 0;
}

// Host-side check of descriptors: ranges inside the j-memory and the
// i-arrays, finite times and softening, no two clusters sharing an i-row.
int check_clusters(Handle *h, int ncl, const g6mi_cluster *cl, int ni_total) {
  if (ncl > 0 && !cl) return fail(h, G6MI_EINVAL, "null cluster array");
  std::vector<std::pair<int, int>> rows;
  rows.reserve(ncl);
  for (int c = 0; c < ncl; ++c) {
    const g6mi_cluster &d = cl[c];
    const std::string at = "cluster " + std::to_string(c) + ": ";
    if (d.joff < 0 || d.nj < 0 || static_cast<long long>(d.joff) + d.nj > static_cast<long long>(h->n_contig))
      return fail(h, G6MI_EINVAL, at + "j-slots outside the slots set from slot 0");
    if (d.ioff < 0 || d.ni < 0 || static_cast<long long>(d.ioff) + d.ni > ni_total)
      return fail(h, G6MI_EINVAL, at + "i-rows outside 0 .. ni_total-1");
    if (!std::isfinite(d.ti) || !std::isfinite(d.eps2) || d.eps2 < 0.0)
      return fail(h, G6MI_EINVAL, at + "ti and eps2 must be finite, eps2 >= 0");
    if (d.ni > 0) rows.emplace_back(d.ioff, d.ioff + d.ni);
  }
  std::sort(rows.begin(), rows.end());
  for (size_t k = 1; k < rows.size(); ++k)
    if (rows[k].first < rows[k - 1].second) return fail(h, G6MI_EINVAL, "clusters share i-rows");
  return 0;
}

// Copy host descriptors to the handle's device buffer on stream s.
int upload_clusters(Handle &h, int ncl, const g6mi_cluster *cl, hipStream_t s) {
  const size_t bytes = std::max(ncl, 1) * sizeof(g6mi_cluster);
  if (h.cl_busy) {
    HIPCHK(&h, hipEventSynchronize(h.cl_ev));
    h.cl_busy = false;
  }
  HIPCHK(&h, ensure(h.h_cl, bytes));
  HIPCHK(&h, ensure(h.d_cl, bytes));
  if (!h.cl_ev) HIPCHK(&h, hipEventCreateWithFlags(&h.cl_ev, hipEventDisableTiming));
  if (ncl > 0) std::memcpy(h.h_cl.p, cl, ncl * sizeof(g6mi_cluster));
  HIPCHK(&h, hipMemcpyAsync(h.d_cl.p, h.h_cl.p, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(&h, hipEventRecord(h.cl_ev, s));
  h.cl_busy = true;
  return 0;
}

} // namespace

// =========================================================== exported ABI

G6MI_API int g6_open(int id) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (id < 0 || id >= G6MI_MAX_HANDLES) return fail(nullptr, G6MI_EINVAL, "invalid handle id");
  Handle &h = g_h[id];
  if (h.open) return fail(&h, G6MI_ESTATE, "handle already open");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(&h, G6MI_EDEVICE, "no HIP device available");
  }
  int dev = 0;
  if (const char *s = std::getenv("G6MI_DEVICE")) dev = std::atoi(s);
  else if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (dev < 0 || dev >= ndev) return fail(&h, G6MI_EDEVICE, "G6MI_DEVICE out of range");
  h = Handle{};
  h.device = dev;
  HIPCHK(&h, hipSetDevice(dev));
  hipDeviceProp_t prop;
  HIPCHK(&h, hipGetDeviceProperties(&prop, dev));
  h.ncu = prop.multiProcessorCount;
  h.clock_mhz = prop.clockRate / 1000;
  h.arch = prop.gcnArchName;
  HIPCHK(&h, hipStreamCreateWithFlags(&h.stream, hipStreamNonBlocking));
  HIPCHK(&h, hipEventCreateWithFlags(&h.stage_ev, hipEventDisableTiming));
  h.prec = parse_precision(std::getenv("G6MI_PRECISION"), G6MI_PREC_DS);
  h.open = true;
  return G6MI_OK;
}

G6MI_API int g6_close(int id) {
  std::lock_guard<std::mutex> lk(g_mu);
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->c_stream && h->c_stream != h->stream) (void)hipStreamSynchronize(h->c_stream);
  destroy_graph(*h);
  if (h->hs.exec) (void)hipGraphExecDestroy(h->hs.exec);
  if (h->hs.graph) (void)hipGraphDestroy(h->hs.graph);
  for (DevBuf *b : {&h->hs.d_ctl, &h->hs.d_state, &h->hs.d_block}) b->release();
  h->hs.h_ctl.release();
  for (DevBuf *b : {&h->d_jm, &h->d_pred, &h->d_stage, &h->d_i, &h->d_out, &h->d_part,
                    &h->d_nnr2, &h->d_nnslot, &h->d_nbcount, &h->d_nblist, &h->d_flags,
                    &h->d_ovf, &h->d_cl, &h->d_plan, &h->d_items, &h->d_bwork, &h->d_ibcl, &h->d_sp})
    b->release();
  for (PinBuf *b : {&h->h_stage, &h->h_i, &h->h_out, &h->h_cl}) b->release();
  if (h->cl_ev) (void)hipEventDestroy(h->cl_ev);
  for (auto &q : h->evs)
    for (auto &ev : q) (void)hipEventDestroy(ev);
  if (h->stage_ev) (void)hipEventDestroy(h->stage_ev);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  *h = Handle{};
  return G6MI_OK;
}

G6MI_API int g6_npipes(void) {
  if (const char *s = std::getenv("G6MI_NPIPES")) {
    const long v = std::atol(s);
    if (v >= 1 && v <= G6MI_NI_MAX) return static_cast<int>(v);
  }
  return G6MI_NPIPES_DEFAULT;
}

G6MI_API void g6_set_tunit(int) {}
G6MI_API void g6_set_xunit(int) {}

namespace {
int check_j(Handle *h, int address, double tj, double mass, const double *j6, const double *a2,
            const double *v, const double *x) {
  if (address < 0 || address >= G6MI_NJ_MAX) return fail(h, G6MI_EINVAL, "address out of range");
  if (!j6 || !a2 || !v || !x) return fail(h, G6MI_EINVAL, "null j-particle array");
  if (!std::isfinite(tj) || !std::isfinite(mass) || !finite3(x) || !finite3(v) || !finite3(a2) ||
      !finite3(j6))
    return fail(h, G6MI_EINVAL, "non-finite j-particle data");
  return 0;
}

// Stage one checked record in the host master copy (uploaded by the next
// calculation).
void store_j(Handle *h, int address, int index, double tj, double mass, const double *j6,
             const double *a2, const double *v, const double *x) {
  grow_host(*h, static_cast<size_t>(address) + 1);
  double *r = &h->h_rec[static_cast<size_t>(address) * kRecDoubles];
  r[0] = tj;
  r[1] = mass;
  for (int d = 0; d < 3; ++d) {
    r[2 + d] = x[d];
    r[5 + d] = v[d];
    r[8 + d] = a2[d];
    r[11 + d] = j6[d];
  }
  r[14] = static_cast<double>(index);
  r[15] = 0.0;
  const int old = h->h_index[address];
  if (old != index) {
    auto it = h->slot_of.find(old);
    if (old >= 0 && it != h->slot_of.end() && it->second == address) h->slot_of.erase(it);
  }
  h->h_index[address] = index;
  h->slot_of[index] = address;
  h->h_set[address] = 1;
  while (h->n_contig < h->h_set.size() && h->h_set[h->n_contig]) ++h->n_contig;
  mark_dirty(*h, address);
}
} // namespace

G6MI_API int g6_set_j_particle(int id, int address, int index, double tj, double dtj,
                               double mass, const double k18[3], const double j6[3],
                               const double a2[3], const double v[3], const double x[3]) {
  (void)dtj;
  (void)k18;
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  const int rc = check_j(h, address, tj, mass, j6, a2, v, x);
  if (rc) return rc;
  store_j(h, address, index, tj, mass, j6, a2, v, x);
  return G6MI_OK;
}

G6MI_API int g6mi_set_j_particles(int id, int n, const int address[], const int index[],
                                  const double tj[], const double dtj[], const double mass[],
                                  const double j6[][3], const double a2[][3], const double v[][3],
                                  const double x[][3]) {
  (void)dtj;
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (n < 0) return fail(h, G6MI_EINVAL, "negative record count");
  if (n > 0 && (!address || !index || !tj || !mass || !j6 || !a2 || !v || !x))
    return fail(h, G6MI_EINVAL, "null j-particle array");
  for (int k = 0; k < n; ++k) {
    const int rc = check_j(h, address[k], tj[k], mass[k], j6[k], a2[k], v[k], x[k]);
    if (rc) return rc;
  }
  for (int k = 0; k < n; ++k) store_j(h, address[k], index[k], tj[k], mass[k], j6[k], a2[k], v[k], x[k]);
  return G6MI_OK;
}

G6MI_API void g6_set_ti(int id, double ti) {
  Handle *h = get_open(id);
  if (h) h->ti = ti;
}

G6MI_API int g6calc_firsthalf(int id, int nj, int ni, const int index[], const double xi[][3],
                              const double vi[][3], const double aold[][3],
                              const double j6old[][3], const double phiold[], double eps2,
                              const double h2[]) {
  (void)aold;
  (void)j6old;
  (void)phiold;
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (h->pending && !h->pending_err) (void)hipStreamSynchronize(h->stream); // superseded
  h->pending = true;
  h->res_valid = false;
  h->c_have = false;
  hipError_t e = hipSetDevice(h->device);
  int rc = e == hipSuccess ? firsthalf_impl(*h, nj, ni, index, xi, vi, eps2, h2)
                           : hip_fail(h, e, "hipSetDevice");
  h->pending_err = rc;
  return rc;
}

G6MI_API int g6calc_lasthalf(int id, int nj, int ni, const int index[], const double xi[][3],
                             const double vi[][3], double eps2, const double h2[],
                             double acc[][3], double jerk[][3], double pot[]) {
  (void)xi;
  (void)vi;
  (void)h2;
  return lasthalf_impl(id, nj, ni, index, eps2, acc, jerk, pot, nullptr);
}

G6MI_API int g6calc_lasthalf2(int id, int nj, int ni, const int index[], const double xi[][3],
                              const double vi[][3], double eps2, const double h2[],
                              double acc[][3], double jerk[][3], double pot[],
                              int nnbindex[]) {
  (void)xi;
  (void)vi;
  (void)h2;
  return lasthalf_impl(id, nj, ni, index, eps2, acc, jerk, pot, nnbindex);
}

G6MI_API int g6_nearest_neighbour(int id, int ni, int nnbindex[], double r2nn[]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!h->res_valid) {
    // device-path calculation: fetch the nearest neighbours from its buffers
    return fail(h, G6MI_ESTATE, "no completed host-path calculation");
  }
  if (ni != h->c_ni) return fail(h, G6MI_EINVAL, "ni differs from the last calculation");
  for (int i = 0; i < ni; ++i) {
    if (nnbindex) nnbindex[i] = h->r_nnb[i];
    if (r2nn) r2nn[i] = h->r_r2nn[i];
  }
  return G6MI_OK;
}

G6MI_API int g6_read_neighbour_list(int id) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!h->c_have || h->pending) return fail(h, G6MI_ESTATE, "no completed calculation");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->c_stream));
  const size_t n = static_cast<size_t>(h->c_ni);
  if (n > 0 && h->c_nbl) {
    // overflowed lists: keep the G6MI_NB_MAX smallest indices (exact pass)
    int status[kStatusWords] = {0, 0};
    HIPCHK(h, hipMemcpy(status, h->c_batch ? h->c_bargs.status : h->c_flags, sizeof(status),
                        hipMemcpyDeviceToHost));
    if (status[kStatusOverflowCount] > 0 && !h->nb_exact_done) {
      if (h->c_batch)
        HIPCHK(h, launch_batch_nb_exact(h->c_prec, h->c_bargs, status[kStatusOverflowCount], h->c_stream));
      else if (h->c_fused)
        HIPCHK(h, launch_nb_exact_fused(h->c_prec, h->c_args, h->jm, h->c_ti, h->c_flags, h->c_ovf,
                                        status[kStatusOverflowCount], h->c_stream));
      else
        HIPCHK(h, launch_nb_exact(h->c_prec, h->c_args, h->jm.index, h->c_flags, h->c_ovf,
                                  status[kStatusOverflowCount], h->c_stream));
      HIPCHK(h, hipStreamSynchronize(h->c_stream));
      h->nb_exact_done = true;
    }
  }
  h->r_nbcount.assign(n, 0);
  h->r_nblist.assign(n * kNbMax, -1);
  if (n > 0) {
    const ForceArgs &ca = h->c_batch ? h->c_bargs.fa : h->c_args;
    HIPCHK(h, hipMemcpy(h->r_nbcount.data(), ca.nb_count, n * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(h->r_nblist.data(), ca.nb_slot, n * kNbMax * sizeof(int), hipMemcpyDeviceToHost));
  }
  h->nb_read = true;
  bool over = false;
  for (size_t i = 0; i < n; ++i) over = over || h->r_nbcount[i] > kNbMax;
  return over ? G6MI_WARN : G6MI_OK;
}

G6MI_API int g6_get_neighbour_list(int id, int ipipe, int maxlength, int *nblen, int nbl[]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!h->nb_read) return fail(h, G6MI_ESTATE, "g6_read_neighbour_list was not called");
  if (ipipe < 0 || ipipe >= h->c_ni || maxlength < 0 || !nblen || (maxlength > 0 && !nbl))
    return fail(h, G6MI_EINVAL, "bad neighbour-list request");
  const int cnt = h->r_nbcount[ipipe];
  const int k = std::min(std::min(cnt, maxlength), kNbMax);
  std::memcpy(nbl, &h->r_nblist[static_cast<size_t>(ipipe) * kNbMax], sizeof(int) * k);
  *nblen = cnt;
  return cnt > k ? G6MI_WARN : G6MI_OK;
}

G6MI_API const char *g6mi_last_error(int id) {
  if (id < 0 || id >= G6MI_MAX_HANDLES) return g_err.c_str();
  return g_h[id].err.c_str();
}

G6MI_API int g6mi_nb_max(void) { return G6MI_NB_MAX; }

G6MI_API int g6mi_set_precision(int id, int prec) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (prec != G6MI_PREC_FP32 && prec != G6MI_PREC_DS && prec != G6MI_PREC_FP64)
    return fail(h, G6MI_EINVAL, "unknown precision variant");
  h->prec = prec;
  return G6MI_OK;
}

G6MI_API int g6mi_get_precision(int id) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  return h->prec;
}

G6MI_API int g6mi_set_neighbour_lists(int id, int on) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  h->nbl = on != 0;
  return G6MI_OK;
}

G6MI_API int g6mi_set_spatial(int id, int mode) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (mode < 0 || mode > 2) return fail(h, G6MI_EINVAL, "spatial mode must be 0, 1 or 2");
  h->spatial = mode;
  return G6MI_OK;
}

G6MI_API int g6mi_calc_device_noalloc(int id, int nj, int ni, const int *d_islot, const double *d_xi,
                                      const double *d_vi, double eps2, const double *d_h2,
                                      double *d_acc, double *d_jerk, double *d_pot, int *d_nnb,
                                      double *d_r2nn, void *stream) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (h->pending) return fail(h, G6MI_ESTATE, "a host-path calculation is pending");
  if (nj < 0 || static_cast<size_t>(nj) > h->n_contig)
    return fail(h, G6MI_EINVAL, "nj exceeds the number of j-slots set from slot 0");
  if (ni < 0 || ni > G6MI_NI_MAX) return fail(h, G6MI_EINVAL, "ni out of range");
  if (ni > 0 && (!d_islot || !d_xi || !d_vi || !d_h2 || !d_acc || !d_jerk || !d_pot))
    return fail(h, G6MI_EINVAL, "null device array");
  if (!std::isfinite(eps2) || eps2 < 0.0) return fail(h, G6MI_EINVAL, "eps2 must be finite and >= 0");
  if (!h->jm.t || static_cast<size_t>(std::max(nj, 1)) > h->jm.cap)
    return fail(h, G6MI_ESTATE, "the device j-memory holds fewer than nj slots");
  HIPCHK(h, hipSetDevice(h->device));
  void *scr = nullptr;
  size_t scr_bytes = 0;
  HIPCHK(h, scratch_region(h->device, &scr, &scr_bytes));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  h->res_valid = false;
  return enqueue_calc(*h, nj, ni, d_islot, d_xi, d_vi, d_h2, eps2, d_acc, d_jerk, d_pot, d_nnb, d_r2nn, s,
                      scr, scr_bytes);
}

G6MI_API int g6mi_set_fused_predict(int id, int on) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (on != 0 && on != 1) return fail(h, G6MI_EINVAL, "fused prediction flag must be 0 or 1");
  h->fuse = on != 0;
  return G6MI_OK;
}

G6MI_API int g6mi_set_shape(int id, int i_per_group, int j_splits) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (i_per_group < 0 || i_per_group > 2 * kWG || (i_per_group & (i_per_group - 1)) ||
      j_splits < 0 || j_splits > 4096)
    return fail(h, G6MI_EINVAL, "bad launch shape");
  h->user_ipw = i_per_group;
  h->user_nsplit = j_splits;
  return G6MI_OK;
}

G6MI_API int g6mi_get_shape(int id, int shape[4]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!shape) return fail(h, G6MI_EINVAL, "null shape");
  for (int q = 0; q < 4; ++q) shape[q] = h->shape[q];
  return G6MI_OK;
}

G6MI_API int g6mi_enable_timing(int id, int on) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  h->timing = on != 0;
  h->n_timed = 0;
  return G6MI_OK;
}

namespace {
int timing_of(Handle *h, int k, double ms[3]) {
  HIPCHK(h, hipEventSynchronize(h->evs[k][3]));
  for (int q = 0; q < 3; ++q) {
    float t = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&t, h->evs[k][q], h->evs[k][q + 1]));
    ms[q] = t;
  }
  return 0;
}
} // namespace

G6MI_API int g6mi_last_timing(int id, double ms[3]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!ms) return fail(h, G6MI_EINVAL, "null ms");
  if (h->n_timed == 0) return fail(h, G6MI_ESTATE, "no timed calculation");
  HIPCHK(h, hipSetDevice(h->device));
  return timing_of(h, h->n_timed - 1, ms);
}

G6MI_API int g6mi_timing_totals(int id, double ms[3], int *count) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!ms || !count) return fail(h, G6MI_EINVAL, "null argument");
  HIPCHK(h, hipSetDevice(h->device));
  ms[0] = ms[1] = ms[2] = 0.0;
  for (int k = 0; k < h->n_timed; ++k) {
    double one[3];
    int rc = timing_of(h, k, one);
    if (rc) return rc;
    for (int q = 0; q < 3; ++q) ms[q] += one[q];
  }
  *count = h->n_timed;
  h->n_timed = 0;
  return G6MI_OK;
}

G6MI_API int g6mi_set_j_particles_device(int id, int nj, const double *d_t, const double *d_mass,
                                         const int *d_index, const double *d_x,
                                         const double *d_v, const double *d_a2,
                                         const double *d_j6, void *stream) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (nj < 0 || nj > G6MI_NJ_MAX) return fail(h, G6MI_EINVAL, "nj out of range");
  if (nj > 0 && (!d_t || !d_mass || !d_index || !d_x || !d_v || !d_a2 || !d_j6))
    return fail(h, G6MI_EINVAL, "null device array");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  // the host master must stay authoritative: bring it in sync first
  grow_host(*h, std::max(1, nj));
  int rc = ensure_jmem(*h, std::max<size_t>(h->h_set.size(), static_cast<size_t>(std::max(nj, 1))));
  if (rc) return rc;
  rc = upload_dirty(*h, h->stream);
  if (rc) return rc;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (s != h->stream) HIPCHK(h, hipStreamSynchronize(s));
  HIPCHK(h, launch_load(nj, d_t, d_mass, d_index, d_x, d_v, d_a2, d_j6, h->jm, s));
  // mirror the new records into the host master copy
  std::vector<double> tmp(static_cast<size_t>(nj) * 3);
  std::vector<double> col(static_cast<size_t>(nj));
  std::vector<int> idx(static_cast<size_t>(nj));
  HIPCHK(h, hipStreamSynchronize(s));
  if (nj > 0) {
    HIPCHK(h, hipMemcpy(idx.data(), h->jm.index, sizeof(int) * nj, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(col.data(), h->jm.t, sizeof(double) * nj, hipMemcpyDeviceToHost));
    for (int k = 0; k < nj; ++k) h->h_rec[static_cast<size_t>(k) * kRecDoubles + 0] = col[k];
    HIPCHK(h, hipMemcpy(col.data(), h->jm.m, sizeof(double) * nj, hipMemcpyDeviceToHost));
    for (int k = 0; k < nj; ++k) h->h_rec[static_cast<size_t>(k) * kRecDoubles + 1] = col[k];
    const double *srcs[4] = {h->jm.x, h->jm.v, h->jm.a2, h->jm.j6};
    for (int f = 0; f < 4; ++f)
      for (int d = 0; d < 3; ++d) {
        HIPCHK(h, hipMemcpy(col.data(), srcs[f] + d * h->jm.cap, sizeof(double) * nj,
                            hipMemcpyDeviceToHost));
        for (int k = 0; k < nj; ++k)
          h->h_rec[static_cast<size_t>(k) * kRecDoubles + 2 + 3 * f + d] = col[k];
      }
  }
  for (int k = 0; k < nj; ++k) {
    const int old = h->h_index[k];
    auto it = h->slot_of.find(old);
    if (old >= 0 && it != h->slot_of.end() && it->second == k) h->slot_of.erase(it);
  }
  for (int k = 0; k < nj; ++k) {
    h->h_rec[static_cast<size_t>(k) * kRecDoubles + 14] = static_cast<double>(idx[k]);
    h->h_index[k] = idx[k];
    h->slot_of[idx[k]] = k;
    h->h_set[k] = 1;
  }
  while (h->n_contig < h->h_set.size() && h->h_set[h->n_contig]) ++h->n_contig;
  return G6MI_OK;
}

G6MI_API int g6mi_calc_device(int id, int nj, int ni, const int *d_islot, const double *d_xi,
                              const double *d_vi, double eps2, const double *d_h2,
                              double *d_acc, double *d_jerk, double *d_pot, int *d_nnb,
                              double *d_r2nn, void *stream) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (h->pending) return fail(h, G6MI_ESTATE, "a host-path calculation is pending");
  if (nj < 0 || static_cast<size_t>(nj) > h->n_contig)
    return fail(h, G6MI_EINVAL, "nj exceeds the number of j-slots set from slot 0");
  if (ni < 0 || ni > G6MI_NI_MAX) return fail(h, G6MI_EINVAL, "ni out of range");
  if (ni > 0 && (!d_islot || !d_xi || !d_vi || !d_h2 || !d_acc || !d_jerk || !d_pot))
    return fail(h, G6MI_EINVAL, "null device array");
  if (!std::isfinite(eps2) || eps2 < 0.0) return fail(h, G6MI_EINVAL, "eps2 must be finite and >= 0");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  int rc = ensure_jmem(*h, std::max<size_t>(1, static_cast<size_t>(nj)));
  if (rc) return rc;
  h->res_valid = false;
  return enqueue_calc(*h, nj, ni, d_islot, d_xi, d_vi, d_h2, eps2, d_acc, d_jerk, d_pot, d_nnb,
                      d_r2nn, s);
}

G6MI_API int g6mi_last_status(int id, int *flags) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!flags) return fail(h, G6MI_EINVAL, "null flags");
  if (!h->c_have || h->pending) return fail(h, G6MI_ESTATE, "no completed calculation");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->c_stream));
  int st[kStatusWords] = {0, 0};
  HIPCHK(h, hipMemcpy(st, h->c_batch ? h->c_bargs.status : h->c_flags, sizeof(st), hipMemcpyDeviceToHost));
  *flags = st[kStatusFlags];
  return G6MI_OK;
}

// ------------------------------------------------------------ batched calls

G6MI_API int g6mi_batch_calc_device(int id, int ncl, const g6mi_cluster *d_cl, int ni_total,
                                    const int *d_islot, const double *d_xi, const double *d_vi,
                                    const double *d_h2, double *d_acc, double *d_jerk,
                                    double *d_pot, int *d_nnb, double *d_r2nn, void *stream) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  int rc = check_batch_args(h, ncl, ni_total, d_islot, d_xi, d_vi, d_h2, d_acc, d_jerk, d_pot);
  if (rc) return rc;
  if (ncl > 0 && !d_cl) return fail(h, G6MI_EINVAL, "null cluster array");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  return enqueue_batch(*h, ncl, d_cl, ni_total, d_islot, d_xi, d_vi, d_h2, d_acc, d_jerk, d_pot,
                       d_nnb, d_r2nn, s);
}

G6MI_API int g6mi_batch_calc(int id, int ncl, const g6mi_cluster *cl, int ni_total,
                             const int *d_islot, const double *d_xi, const double *d_vi,
                             const double *d_h2, double *d_acc, double *d_jerk, double *d_pot,
                             int *d_nnb, double *d_r2nn, void *stream) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  int rc = check_batch_args(h, ncl, ni_total, d_islot, d_xi, d_vi, d_h2, d_acc, d_jerk, d_pot);
  if (!rc) rc = check_clusters(h, ncl, cl, ni_total);
  if (rc) return rc;
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  rc = upload_clusters(*h, ncl, cl, s);
  if (rc) return rc;
  return enqueue_batch(*h, ncl, static_cast<const g6mi_cluster *>(h->d_cl.p), ni_total, d_islot, d_xi,
                       d_vi, d_h2, d_acc, d_jerk, d_pot, d_nnb, d_r2nn, s);
}

G6MI_API int g6mi_batch_use_graph(int id, int on) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  h->use_graph = on != 0;
  if (!h->use_graph) {
    HIPCHK(h, hipSetDevice(h->device));
    if (h->c_stream) HIPCHK(h, hipStreamSynchronize(h->c_stream));
    destroy_graph(*h);
  }
  return G6MI_OK;
}

namespace {
int check_tuning(Handle *h, const g6mi_batch_tuning *t) {
  if (t->item_work < 1 || t->item_work > 1024 || t->wide_min < 1 || t->wg_per_cu < 0 || t->wg_per_cu > 8 ||
      t->max_split < 1 || t->max_split > 4096)
    return fail(h, G6MI_EINVAL, "tuning out of range");
  return 0;
}

void apply_tuning(Handle &h, const g6mi_batch_tuning &t) {
  h.btune.item_work = t.item_work;
  h.btune.wide_min = t.wide_min;
  h.btune.max_split = t.max_split;
  h.b_wg_per_cu = t.wg_per_cu;
}

g6mi_batch_tuning current_tuning(const Handle &h) {
  g6mi_batch_tuning t;
  t.item_work = h.btune.item_work;
  t.wide_min = h.btune.wide_min;
  t.max_split = h.btune.max_split;
  t.wg_per_cu = h.b_wg_per_cu;
  return t;
}

// Tuning results of this process, by workload key.
std::mutex g_tune_mu;
std::unordered_map<std::string, g6mi_batch_tuning> g_tune;

constexpr const char *kTuneTag = "g6mi-batch-tune-v2";

int ilog2_floor(double v) { return v >= 1.0 ? static_cast<int>(std::floor(std::log2(v))) : -1; }

// Workload key: device, variant, and the batch's size class (number of
// clusters, log2 of pairs, i-particles and j-slots).
std::string tune_key(const Handle &h, int ncl, const g6mi_cluster *cl) {
  double pairs = 0.0, nj = 0.0, ni = 0.0;
  for (int c = 0; c < ncl; ++c) {
    pairs += static_cast<double>(cl[c].ni) * cl[c].nj;
    nj += cl[c].nj;
    ni += cl[c].ni;
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/cu%d/p%d/nb%d/c%d/lp%d/li%d/lj%d", h.arch.empty() ? "gpu" : h.arch.c_str(),
                h.ncu, h.prec, h.nbl ? 1 : 0, ncl, ilog2_floor(pairs), ilog2_floor(ni), ilog2_floor(nj));
  std::string k(buf);
  for (char &ch : k)
    if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
  return k;
}

bool cache_lookup(const char *path, const std::string &key, g6mi_batch_tuning &t) {
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      t = it->second;
      return true;
    }
  }
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    char tag[64], k[512];
    g6mi_batch_tuning v;
    double ms = 0.0;
    if (std::sscanf(line, "%63s %511s %d %d %d %d %lf", tag, k, &v.item_work, &v.wide_min, &v.wg_per_cu,
                    &v.max_split, &ms) == 7 &&
        key == k && std::string(tag) == kTuneTag) {
      t = v; // the last entry for the key wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}
} // namespace

G6MI_API int g6mi_batch_set_tuning(int id, const g6mi_batch_tuning *t) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  g6mi_batch_tuning v;
  if (t) {
    int rc = check_tuning(h, t);
    if (rc) return rc;
    v = *t;
  } else {
    BatchTune d;
    v.item_work = d.item_work;
    v.wide_min = d.wide_min;
    v.max_split = d.max_split;
    v.wg_per_cu = 0;
  }
  apply_tuning(*h, v);
  return G6MI_OK;
}

G6MI_API int g6mi_batch_get_tuning(int id, g6mi_batch_tuning *t) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!t) return fail(h, G6MI_EINVAL, "null tuning");
  *t = current_tuning(*h);
  return G6MI_OK;
}

G6MI_API int g6mi_batch_autotune(int id, int ncl, const g6mi_cluster *cl, int ni_total,
                                 const int *d_islot, const double *d_xi, const double *d_vi,
                                 const double *d_h2, double *d_acc, double *d_jerk, double *d_pot,
                                 int *d_nnb, double *d_r2nn, void *stream, const char *cache_path,
                                 int reps, g6mi_batch_tuning *best) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  int rc = check_batch_args(h, ncl, ni_total, d_islot, d_xi, d_vi, d_h2, d_acc, d_jerk, d_pot);
  if (!rc) rc = check_clusters(h, ncl, cl, ni_total);
  if (rc) return rc;
  if (!cache_path) cache_path = std::getenv("G6MI_TUNE_CACHE");
  const std::string key = tune_key(*h, ncl, cl);
  g6mi_batch_tuning found;
  if (cache_lookup(cache_path, key, found) && check_tuning(h, &found) == 0) {
    apply_tuning(*h, found);
    if (best) *best = found;
    return G6MI_OK;
  }
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : h->stream;
  rc = upload_clusters(*h, ncl, cl, s);
  if (rc) return rc;
  const g6mi_cluster *d_cl = static_cast<const g6mi_cluster *>(h->d_cl.p);
  if (reps <= 0) reps = 3;
  const bool graph = h->use_graph, timing = h->timing;
  h->use_graph = false;
  h->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const g6mi_batch_tuning base = current_tuning(*h);
  g6mi_batch_tuning win = base;
  double win_ms = INFINITY;
  for (int iw : {1, 2, 4, 8, 16, 32, 64})
    for (int wm : {257, 512, 1024, 1 << 30})
      for (int wg = 1; wg <= batch_waves(h->prec, wm > ni_total) && rc == 0; ++wg) {
        g6mi_batch_tuning t = base;
        t.item_work = iw;
        t.wide_min = wm;
        t.wg_per_cu = wg;
        apply_tuning(*h, t);
        for (int r = 0; r <= reps && rc == 0; ++r) { // one untimed run, then reps timed
          if (r == 1 && hipEventRecord(e0, s) != hipSuccess) rc = fail(h, G6MI_EDEVICE, "event");
          if (!rc)
            rc = enqueue_batch(*h, ncl, d_cl, ni_total, d_islot, d_xi, d_vi, d_h2, d_acc, d_jerk, d_pot, d_nnb,
                               d_r2nn, s);
        }
        if (rc) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(h, G6MI_EDEVICE, "autotune timing");
          break;
        }
        const double per = ms / reps;
        if (per < win_ms) {
          win_ms = per;
          win = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->use_graph = graph;
  h->timing = timing;
  if (rc) {
    apply_tuning(*h, base);
    return rc;
  }
  apply_tuning(*h, win);
  if (best) *best = win;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = win;
  }
  if (cache_path) {
    FILE *f = std::fopen(cache_path, "a");
    if (!f) return fail(h, G6MI_WARN, std::string("cannot append to tuning cache ") + cache_path);
    std::fprintf(f, "%s %s %d %d %d %d %.6f\n", kTuneTag, key.c_str(), win.item_work, win.wide_min,
                 win.wg_per_cu, win.max_split, win_ms);
    std::fclose(f);
  }
  return G6MI_OK;
}

// ------------------------------------------------ device-resident block steps

namespace {
void hs_destroy_graph(Handle &h) {
  if (h.hs.exec) (void)hipGraphExecDestroy(h.hs.exec);
  if (h.hs.graph) (void)hipGraphDestroy(h.hs.graph);
  h.hs.exec = nullptr;
  h.hs.graph = nullptr;
  h.hs.key.clear();
}

// Batch arguments of the current block (descriptor in the control block).
int hs_batch(Handle &h, BatchArgs &b) {
  HermiteArgs &a = h.hs.a;
  const int n = h.hs.n;
  int *nnb = reinterpret_cast<int *>(a.pot1 + 2 * static_cast<size_t>(n));
  return prepare_batch(h, 1, &a.ctl->desc, n, n, a.active, a.xi, a.vi, a.h2i, a.acc1, a.jrk1, a.pot1, nnb,
                       a.pot1 + n, b);
}

int hs_read_ctl(Handle &h, hipStream_t s, HermiteCtl &c) {
  HIPCHK(&h, hipMemcpyAsync(h.hs.h_ctl.p, h.hs.a.ctl, sizeof(HermiteCtl), hipMemcpyDeviceToHost, s));
  HIPCHK(&h, hipStreamSynchronize(s));
  std::memcpy(&c, h.hs.h_ctl.p, sizeof(HermiteCtl));
  return 0;
}
} // namespace

// Order key of a double, as the device kernels map block times onto
// unsigned 64-bit keys (a larger double gives a larger key).
uint64_t order_key_host(double x) {
  uint64_t b;
  std::memcpy(&b, &x, sizeof(b));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

G6MI_API int g6mi_hermite_init(int id, int n, double eps2, double h2, double eta, double eta_s, double dt_max,
                               double dt_min) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (h->pending) return fail(h, G6MI_ESTATE, "a host-path calculation is pending");
  if (n < 1 || static_cast<size_t>(n) > h->n_contig)
    return fail(h, G6MI_EINVAL, "n must be 1 .. the number of j-slots set from slot 0");
  if (!std::isfinite(eps2) || eps2 < 0.0 || !std::isfinite(h2) || !(eta > 0.0) || !std::isfinite(eta) ||
      !(eta_s > 0.0) || !std::isfinite(eta_s) || !(dt_min > 0.0) || !(dt_max >= dt_min) || !std::isfinite(dt_max))
    return fail(h, G6MI_EINVAL, "bad integrator parameters");
  const double t0 = h->h_rec[0];
  for (int k = 1; k < n; ++k)
    if (h->h_rec[static_cast<size_t>(k) * kRecDoubles] != t0)
      return fail(h, G6MI_EINVAL, "the particles must share one time to start");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  int rc = ensure_jmem(*h, std::max<size_t>(1, h->n_contig));
  if (!rc) rc = upload_dirty(*h, s);
  if (rc) return rc;
  auto &hs = h->hs;
  hs_destroy_graph(*h);
  hs.ready = false;
  const size_t cap = h->jm.cap, nn = static_cast<size_t>(n);
  HIPCHK(h, ensure(hs.d_ctl, sizeof(HermiteCtl)));
  HIPCHK(h, ensure(hs.d_state, 8 * cap * sizeof(double)));
  // block: xi, vi, acc1, jrk1 [n][3]; h2i, pot1, r2nn [n]; nnb, active [n] int
  HIPCHK(h, ensure(hs.d_block, (15 * nn) * sizeof(double) + 2 * nn * sizeof(int)));
  HIPCHK(h, ensure(hs.h_ctl, sizeof(HermiteCtl)));
  HermiteArgs &a = hs.a;
  a = HermiteArgs{};
  a.ctl = static_cast<HermiteCtl *>(hs.d_ctl.p);
  a.jm = h->jm;
  double *st = static_cast<double *>(hs.d_state.p);
  a.acc = st;
  a.jrk = st + 3 * cap;
  a.dt = st + 6 * cap;
  a.pot = st + 7 * cap;
  a.n = n;
  double *blk = static_cast<double *>(hs.d_block.p);
  a.xi = blk;
  a.vi = blk + 3 * nn;
  a.acc1 = blk + 6 * nn;
  a.jrk1 = blk + 9 * nn;
  a.h2i = blk + 12 * nn;
  a.pot1 = blk + 13 * nn; // then r2nn [n] and nnb, active (ints)
  a.active = reinterpret_cast<int *>(blk + 15 * nn) + nn;
  a.eps2 = eps2;
  a.h2 = h2;
  a.eta = eta;
  a.eta_s = eta_s;
  a.dt_max = dt_max;
  a.dt_min = dt_min;
  hs.n = n;
  hs.cap = cap;
  hs.jm_t = h->jm.t;
  HermiteCtl c{};
  // the first block: every particle, due at t0 (steps are zero until the
  // first force evaluation)
  c.key[0] = order_key_host(t0);
  c.key[1] = 0xfff0000000000000ull; // +inf
  c.phase = 0;
  c.t_end = INFINITY;
  c.time = t0;
  c.desc = g6mi_cluster{0, n, 0, 0, t0, eps2};
  std::memcpy(hs.h_ctl.p, &c, sizeof(c));
  HIPCHK(h, hipMemcpyAsync(a.ctl, hs.h_ctl.p, sizeof(c), hipMemcpyHostToDevice, s));
  BatchArgs b;
  rc = hs_batch(*h, b);
  if (rc) return rc;
  HIPCHK(h, launch_hs_reset(a, s));
  HIPCHK(h, launch_hs_select(a, b, s));
  HIPCHK(h, launch_batch_force(h->prec, b, b.grid, s));
  HIPCHK(h, launch_hs_start(a, s));
  rc = hs_read_ctl(*h, s, c);
  if (rc) return rc;
  h->c_have = false; // the work buffers now hold the integrator's block
  hs.ready = true;
  return (c.flags & 1) ? G6MI_WARN : G6MI_OK;
}

G6MI_API int g6mi_hermite_advance(int id, double t_end, long long max_steps, double *t_reached,
                                  long long counts[2]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  auto &hs = h->hs;
  if (!hs.ready) return fail(h, G6MI_ESTATE, "g6mi_hermite_init was not called");
  if (h->pending) return fail(h, G6MI_ESTATE, "a host-path calculation is pending");
  if (h->jm.t != hs.jm_t || h->jm.cap != hs.cap)
    return fail(h, G6MI_ESTATE, "the j-memory was reallocated since g6mi_hermite_init");
  if (!std::isfinite(t_end) || max_steps < 0) return fail(h, G6MI_EINVAL, "bad t_end or max_steps");
  HIPCHK(h, hipSetDevice(h->device));
  hipStream_t s = h->stream;
  int rc = upload_dirty(*h, s);
  if (rc) return rc;
  HermiteArgs &a = hs.a;
  HermiteCtl c;
  std::memcpy(hs.h_ctl.p, &t_end, sizeof(double));
  HIPCHK(h, hipMemcpyAsync(&a.ctl->t_end, hs.h_ctl.p, sizeof(double), hipMemcpyHostToDevice, s));
  BatchArgs b;
  rc = hs_batch(*h, b);
  if (rc) return rc;
  const int grid = b.grid;
  std::vector<uint64_t> key = graph_key(*h, b, grid, s);
  if (!hs.exec || key != hs.key) {
    hs_destroy_graph(*h);
    HIPCHK(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_hs_select(a, b, s);
    if (e == hipSuccess) e = launch_batch_items(h->prec, b, grid, s);
    if (e == hipSuccess) e = launch_hs_correct(a, b, grid, s);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &g);
    if (e == hipSuccess) e = ec;
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(h, e, "block-step graph capture");
    }
    hs.graph = g;
    e = hipGraphInstantiate(&hs.exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hs.exec = nullptr;
      hs_destroy_graph(*h);
      return hip_fail(h, e, "hipGraphInstantiate");
    }
    hs.key = std::move(key);
  }
  // Replays past the last block before t_end select nothing and change
  // nothing, so steps are launched in chunks between checks.
  long long launched = 0;
  bool done = false;
  while (launched < max_steps && !done) {
    const long long chunk = std::min<long long>(32, max_steps - launched);
    for (long long q = 0; q < chunk; ++q) HIPCHK(h, hipGraphLaunch(hs.exec, s));
    launched += chunk;
    rc = hs_read_ctl(*h, s, c);
    if (rc) return rc;
    done = c.done != 0;
  }
  if (launched == 0) {
    rc = hs_read_ctl(*h, s, c);
    if (rc) return rc;
  }
  if (t_reached) *t_reached = c.time;
  if (counts) {
    counts[0] = c.block_steps;
    counts[1] = c.particle_steps;
  }
  h->c_have = false;
  return (c.flags & 1) ? G6MI_WARN : G6MI_OK;
}

G6MI_API int g6mi_hermite_state(int id, int n, double x[][3], double v[][3], double acc[][3],
                                double jerk[][3], double pot[], double t[], double dt[]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  auto &hs = h->hs;
  if (!hs.ready) return fail(h, G6MI_ESTATE, "g6mi_hermite_init was not called");
  if (n < 0 || n > hs.n) return fail(h, G6MI_EINVAL, "n exceeds the integrated particles");
  if (h->jm.t != hs.jm_t || h->jm.cap != hs.cap)
    return fail(h, G6MI_ESTATE, "the j-memory was reallocated since g6mi_hermite_init");
  HIPCHK(h, hipSetDevice(h->device));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (n == 0) return G6MI_OK;
  const HermiteArgs &a = hs.a;
  const size_t cap = hs.cap, nn = static_cast<size_t>(n);
  std::vector<double> col(nn);
  auto get = [&](const double *src) -> int {
    HIPCHK(h, hipMemcpy(col.data(), src, nn * sizeof(double), hipMemcpyDeviceToHost));
    return 0;
  };
  // vectors: component d of slot k at [d * cap + k]; also refresh the host
  // master copy of the j-memory (x, v, a/2, jerk/6, t)
  struct Vec {
    const double *src;
    double (*out)[3];
    int rec;    // offset of the vector in the staged record
    double div; // the record holds value / div (a/2, jerk/6)
  } vecs[4] = {{a.jm.x, x, 2, 1.0}, {a.jm.v, v, 5, 1.0}, {a.acc, acc, 8, 2.0}, {a.jrk, jerk, 11, 6.0}};
  for (const Vec &q : vecs)
    for (int d = 0; d < 3; ++d) {
      int rc = get(q.src + d * cap);
      if (rc) return rc;
      for (size_t k = 0; k < nn; ++k) {
        if (q.out) q.out[k][d] = col[k];
        h->h_rec[k * kRecDoubles + q.rec + d] = col[k] / q.div;
      }
    }
  int rc = get(a.jm.t);
  if (rc) return rc;
  for (size_t k = 0; k < nn; ++k) {
    if (t) t[k] = col[k];
    h->h_rec[k * kRecDoubles] = col[k];
  }
  if (pot) {
    rc = get(a.pot);
    if (rc) return rc;
    std::copy(col.begin(), col.end(), pot);
  }
  if (dt) {
    rc = get(a.dt);
    if (rc) return rc;
    std::copy(col.begin(), col.end(), dt);
  }
  return G6MI_OK;
}

G6MI_API int g6mi_device_info(int id, int info[2]) {
  Handle *h = get_open(id);
  if (!h) return code_for_missing(id);
  if (!info) return fail(h, G6MI_EINVAL, "null info");
  info[0] = h->ncu;
  info[1] = h->clock_mhz;
  return G6MI_OK;
}

// ----------------------------------------------------------- Fortran aliases
G6MI_API int g6_open_(const int *id) { return g6_open(*id); }
G6MI_API int g6_close_(const int *id) { return g6_close(*id); }
G6MI_API int g6_npipes_(void) { return g6_npipes(); }
G6MI_API void g6_set_tunit_(const int *t) { g6_set_tunit(*t); }
G6MI_API void g6_set_xunit_(const int *x) { g6_set_xunit(*x); }
G6MI_API void g6_set_ti_(const int *id, const double *ti) { g6_set_ti(*id, *ti); }
G6MI_API int g6_set_j_particle_(const int *id, const int *address, const int *index,
                                const double *tj, const double *dtj, const double *mass,
                                const double k18[3], const double j6[3], const double a2[3],
                                const double v[3], const double x[3]) {
  return g6_set_j_particle(*id, *address, *index, *tj, *dtj, *mass, k18, j6, a2, v, x);
}
G6MI_API int g6calc_firsthalf_(const int *id, const int *nj, const int *ni, const int index[],
                               const double xi[][3], const double vi[][3],
                               const double aold[][3], const double j6old[][3],
                               const double phiold[], const double *eps2, const double h2[]) {
  return g6calc_firsthalf(*id, *nj, *ni, index, xi, vi, aold, j6old, phiold, *eps2, h2);
}
G6MI_API int g6calc_lasthalf_(const int *id, const int *nj, const int *ni, const int index[],
                              const double xi[][3], const double vi[][3], const double *eps2,
                              const double h2[], double acc[][3], double jerk[][3],
                              double pot[]) {
  return g6calc_lasthalf(*id, *nj, *ni, index, xi, vi, *eps2, h2, acc, jerk, pot);
}
G6MI_API int g6calc_lasthalf2_(const int *id, const int *nj, const int *ni, const int index[],
                               const double xi[][3], const double vi[][3], const double *eps2,
                               const double h2[], double acc[][3], double jerk[][3],
                               double pot[], int nnbindex[]) {
  return g6calc_lasthalf2(*id, *nj, *ni, index, xi, vi, *eps2, h2, acc, jerk, pot, nnbindex);
}
G6MI_API int g6_nearest_neighbour_(const int *id, const int *ni, int nnbindex[], double r2nn[]) {
  return g6_nearest_neighbour(*id, *ni, nnbindex, r2nn);
}
G6MI_API int g6_read_neighbour_list_(const int *id) { return g6_read_neighbour_list(*id); }
G6MI_API int g6_get_neighbour_list_(const int *id, const int *ipipe, const int *maxlength,
                                    int *nblen, int nbl[]) {
  return g6_get_neighbour_list(*id, *ipipe, *maxlength, nblen, nbl);
}
