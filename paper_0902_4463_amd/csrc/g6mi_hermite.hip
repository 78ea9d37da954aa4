// Device-resident block steps of the 4th-order Hermite integrator (the
// client side of the paper's CPU/GPU split, Sec. 2 and 2.1, moved onto the
// GPU): one block step is
//
//   hs_select_kernel   the particles with t_k + dt_k = t_b, predicted to t_b
//                      in float64 (Eq. (1)-(2) with the particle's own
//                      a and jerk); t_b = min_k (t_k + dt_k) was gathered by
//                      the previous step: the others' times here, the
//                      corrected ones' in hs_correct_kernel
//   hs_publish_kernel  the one-cluster descriptor and launch plan that the
//                      batched force kernel reads
//   batch_kernel       forces on the block (g6mi_batch.hip)
//   hs_correct_kernel  the split partials added (the batch reduction), then
//                      the Hermite corrector, Aarseth time step, power-of-two
//                      block quantisation; the corrected particle is written
//                      back into the j-memory (its a/2 and jerk/6 too)
//
// Every launch has a fixed grid and reads the block size from device
// memory, so a whole step is one captured graph, replayed without the host.
// The integrator's formulas follow the host driver (hermite/driver.py) term
// by term, with float contraction switched off so that both round alike.

#include "g6mi_batch_common.h"

namespace g6mi {

// Order-preserving map of doubles onto unsigned 64-bit keys, so that the
// minimum over a grid is one atomicMin.
__device__ __forceinline__ unsigned long long order_key(double x) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double(static_cast<long long>(b));
}
constexpr unsigned long long kKeyInf = 0xfff0000000000000ull; // order_key(+inf)

// Workgroup minimum of one key per thread, folded into *dst with one
// atomic (none when every key is +inf).  Every thread must call it, at most
// once per launch (its LDS words are read after the barrier without a second
// one).
__device__ __forceinline__ void key_min(unsigned long long key, unsigned long long *dst) {
  __shared__ unsigned long long s_key[4];
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(key, off);
    key = o < key ? o : key;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) s_key[wave] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = s_key[0];
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) m = s_key[w] < m ? s_key[w] : m;
    if (m != kKeyInf) atomicMin(dst, m);
  }
}

// Taylor prediction of particle k to time tb from its own a and jerk, the
// host driver's expression: x + tau (v + tau (a/2 + tau j/6)).
__device__ __forceinline__ void predict_particle(const HermiteArgs &h, int k, double tb, double *xp,
                                                 double *vp) {
#pragma clang fp contract(off)
  const double tau = tb - h.jm.t[k];
  for (int d = 0; d < 3; ++d) {
    const size_t e = d * h.jm.cap + k;
    const double a2 = 0.5 * h.acc[e];
    const double j6 = h.jrk[e] / 6.0;
    xp[d] = h.jm.x[e] + tau * (h.jm.v[e] + tau * (a2 + tau * j6));
    vp[d] = h.jm.v[e] + tau * (2.0 * a2 + tau * (3.0 * j6));
  }
}

__global__ __launch_bounds__(256) void hs_select_kernel(HermiteArgs h) {
  __shared__ int s_wave[4], s_base;
  const int tid = threadIdx.x;
  const int k = blockIdx.x * 256 + tid;
  HermiteCtl *ctl = h.ctl;
  // both keys read with the phase, not after it (one dependent load fewer)
  const int ph = ctl->phase;
  const unsigned long long k0 = ctl->key[0], k1 = ctl->key[1];
  const double tb = key_value(ph ? k1 : k0);
  const bool go = tb <= ctl->t_end;
  const double tn = k < h.n ? h.jm.t[k] + h.dt[k] : INFINITY;
  const bool act = go && k < h.n && tn == tb;
  // the active particles' loads go out before the block-wide steps below
  double xp[3], vp[3];
  if (act) predict_particle(h, k, tb, xp, vp);
  // the next block time, first part: the particles this step leaves alone
  key_min(act ? kKeyInf : order_key(tn), &ctl->key[ph ^ 1]);
  // slots of this block's active particles: wave counts, one atomic per block
  const unsigned long long m = __ballot(act);
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) s_wave[wave] = __popcll(m);
  __syncthreads();
  if (tid == 0) {
    const int tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    s_base = tot ? atomicAdd(&ctl->ni_count, tot) : 0;
  }
  __syncthreads();
  if (act) {
    int q = s_base + __popcll(m & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; ++w) q += s_wave[w];
    h.active[q] = k;
    for (int d = 0; d < 3; ++d) {
      h.xi[3 * static_cast<size_t>(q) + d] = xp[d];
      h.vi[3 * static_cast<size_t>(q) + d] = vp[d];
    }
    h.h2i[q] = h.h2;
  }
}

// The block as a one-cluster descriptor for the batched force launch, or an
// empty block once t_b > t_end, so that replays past the end change nothing,
// with the batch's launch plan for that one cluster (the plan kernel's
// decisions for a batch of one: plan_shape, plan_share with the whole grid
// as its share, plan_target, plan_splits) and its work tables; then the
// block-time keys turn over (see HermiteCtl).  A launch of its own after the
// selection: a last-workgroup hand-over inside the selection would need a
// device-scope fence per workgroup, which on gfx950 writes back and
// invalidates the XCD's whole L2.
__global__ __launch_bounds__(256) void hs_publish_kernel(HermiteArgs h, BatchArgs b) {
  __shared__ int s_items, s_nib, s_ni;
  if (threadIdx.x == 0) {
    HermiteCtl *ctl = h.ctl;
    const int ph = ctl->phase;
    const unsigned long long k0 = ctl->key[0], k1 = ctl->key[1];
    const double tb = key_value(ph ? k1 : k0);
    const bool go = tb <= ctl->t_end;
    g6mi_cluster d;
    d.joff = 0;
    d.nj = h.n;
    d.ioff = 0;
    d.ni = go ? ctl->ni_count : 0;
    d.ti = go ? tb : ctl->time;
    d.eps2 = h.eps2;
    ctl->desc = d;
    ctl->done = go ? 0 : 1;
    BatchPlan pl = plan_shape(d.ni, d.nj, b.tune);
    if (pl.nib > 0) plan_share(pl, b.grid, b.tune);
    plan_splits(pl, plan_target(plan_work(pl), b.grid, b.tune), b.tune);
    pl.ib0 = pl.item0 = 0;
    pl.pbase = 0;
    b.plan[0] = pl;
    const int items = pl.nib * pl.nsplit;
    for (int x = 0; x < kQueues; ++x) b.work->head[x] = 0;
    b.work->nitems = min(items, b.item_cap);
    b.work->nib = pl.nib;
    b.status[kStatusFlags] = items > b.item_cap ? kFlagBadCluster : 0;
    b.status[kStatusOverflowCount] = 0;
    s_items = min(items, b.item_cap);
    s_nib = pl.nib;
    s_ni = d.ni;
    // the corrector adds the block's new times to key[ph ^ 1]; the next
    // selection reads it and fills key[ph] afresh
    ctl->ni_count = 0;
    ctl->key[ph] = kKeyInf;
    ctl->phase = ph ^ 1;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < s_items; q += 256) b.item_cl[q] = 0;
  for (int q = threadIdx.x; q < s_nib; q += 256) b.ib_cl[q] = 0;
  if (b.nbl)
    for (int r = threadIdx.x; r < s_ni; r += 256) b.fa.nb_count[r] = 0;
}

__device__ __forceinline__ double norm3(const double *a) {
#pragma clang fp contract(off)
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
}

// Power-of-two step at or below dt, within [dt_min, dt_max]: 2^floor(log2)
// taken exactly from the binary exponent.
__device__ __forceinline__ double quantise(double dt, double dt_min, double dt_max) {
  dt = fmin(fmax(dt, dt_min), dt_max);
  int e;
  (void)frexp(dt, &e); // dt = f 2^e, f in [0.5, 1)
  return ldexp(1.0, e - 1);
}

// Corrector (Makino & Aarseth 1992) for block position q at block time tb,
// given its new force sums f (acc xyz, jerk xyz, sum m/r, as the batch
// reduction wrote them to acc1, jrk1 and pot1 = -f[6]), then the Aarseth
// criterion with the second derivative at the end of the step, and the
// block rule: halve while too long, double only when the time is a multiple
// of the doubled step.  Returns the new step.
__device__ __forceinline__ double correct_particle(const HermiteArgs &h, int q, double tb, const double *f) {
#pragma clang fp contract(off)
  HermiteCtl *ctl = h.ctl;
  const int k = h.active[q];
  const size_t cap = h.jm.cap;
  const double dt = tb - h.jm.t[k];
  double a0[3], j0[3], a1[3], j1[3], a2[3], a3[3], a2e[3];
  bool finite = true;
  for (int d = 0; d < 3; ++d) {
    a0[d] = h.acc[d * cap + k];
    j0[d] = h.jrk[d * cap + k];
    a1[d] = f[d];
    j1[d] = f[3 + d];
    finite = finite && isfinite(a1[d]) && isfinite(j1[d]);
  }
  const double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
  for (int d = 0; d < 3; ++d) {
    a2[d] = (-6.0 * (a0[d] - a1[d]) - dt * (4.0 * j0[d] + 2.0 * j1[d])) / dt2;
    a3[d] = (12.0 * (a0[d] - a1[d]) + 6.0 * dt * (j0[d] + j1[d])) / dt3;
  }
  double xp[3], vp[3];
  for (int d = 0; d < 3; ++d) {
    xp[d] = h.xi[3 * static_cast<size_t>(q) + d];
    vp[d] = h.vi[3 * static_cast<size_t>(q) + d];
  }
  for (int d = 0; d < 3; ++d) {
    const double x1 = xp[d] + a2[d] * dt4 / 24.0 + a3[d] * dt5 / 120.0;
    const double v1 = vp[d] + a2[d] * dt3 / 6.0 + a3[d] * dt4 / 24.0;
    a2e[d] = a2[d] + dt * a3[d];
    h.jm.x[d * cap + k] = x1;
    h.jm.v[d * cap + k] = v1;
    h.acc[d * cap + k] = a1[d];
    h.jrk[d * cap + k] = j1[d];
    h.jm.a2[d * cap + k] = a1[d] / 2.0;
    h.jm.j6[d * cap + k] = j1[d] / 6.0;
  }
  const double na1 = norm3(a1), nj1 = norm3(j1), na3 = norm3(a3), na2e = norm3(a2e);
  const double num = na1 * na2e + nj1 * nj1;
  const double den = nj1 * na3 + na2e * na2e;
  const double dt_new = sqrt(h.eta * num / fmax(den, 1e-300));
  const double old = h.dt[k];
  double nw = old;
  while (dt_new < nw && nw > h.dt_min) nw *= 0.5; // never below dt_min
  if (dt_new >= 2.0 * old && fmod(tb, 2.0 * old) == 0.0 && 2.0 * old <= h.dt_max) nw = 2.0 * old;
  h.jm.t[k] = tb;
  h.dt[k] = nw;
  h.pot[k] = -f[6];
  if (!finite) atomicOr(&ctl->flags, 1);
  return nw;
}

// The block's forces finished from the split partials (reduce_iblock, one
// workgroup per part of an i-block, at most kHsReduceWgs workgroups with
// rows) and each particle corrected by the lane that finished it
// (correct_particle); the minimum of their new t + dt is folded into the
// next block time, one atomic per workgroup with rows.
__global__ __launch_bounds__(256) void hs_correct_kernel(HermiteArgs h, BatchArgs b) {
  HermiteCtl *ctl = h.ctl;
  const int ni = ctl->desc.ni;
  const double tb = ctl->desc.ti;
  if (blockIdx.x == 0 && threadIdx.x == 0 && ni > 0) {
    ctl->block_steps += 1;
    ctl->particle_steps += ni;
    ctl->time = tb;
  }
  unsigned long long next = kKeyInf;
  int fl = 0;
  const int nib_total = b.work->nib;
  const int P = reduce_parts(nib_total, min(static_cast<int>(gridDim.x), kHsReduceWgs), 64);
  for (int u = blockIdx.x; u < nib_total * P; u += gridDim.x)
    fl |= reduce_iblock<true>(b, u / P, u % P, P, [&](int q, const double *sum) {
      const unsigned long long key = order_key(tb + correct_particle(h, q, tb, sum));
      next = key < next ? key : next;
    });
  if (fl) atomicOr(b.status + kStatusFlags, fl);
  // the next block time, second part: this block's particles
  key_min(next, &ctl->key[ctl->phase]);
}

// First step of block position q: a, jerk and potential stored, the step
// eta_s |a| / |jerk| quantised.  Returns the step.
__device__ __forceinline__ double start_particle(const HermiteArgs &h, int q) {
#pragma clang fp contract(off)
  HermiteCtl *ctl = h.ctl;
  const int k = h.active[q];
  const size_t cap = h.jm.cap;
  double a1[3], j1[3];
  bool finite = true;
  for (int d = 0; d < 3; ++d) {
    a1[d] = h.acc1[3 * static_cast<size_t>(q) + d];
    j1[d] = h.jrk1[3 * static_cast<size_t>(q) + d];
    finite = finite && isfinite(a1[d]) && isfinite(j1[d]);
    h.acc[d * cap + k] = a1[d];
    h.jrk[d * cap + k] = j1[d];
    h.jm.a2[d * cap + k] = a1[d] / 2.0;
    h.jm.j6[d * cap + k] = j1[d] / 6.0;
  }
  const double dt = h.eta_s * norm3(a1) / fmax(norm3(j1), 1e-300);
  const double step = quantise(dt, h.dt_min, h.dt_max);
  h.dt[k] = step;
  h.pot[k] = h.pot1[q];
  if (!finite) atomicOr(&ctl->flags, 1);
  return step;
}

// First force evaluation of every particle at the common start time
// (start_particle, one thread each) and the first next block time.
__global__ __launch_bounds__(256) void hs_start_kernel(HermiteArgs h) {
  HermiteCtl *ctl = h.ctl;
  const int ni = ctl->desc.ni;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctl->time = ctl->desc.ti;
  if (blockIdx.x * 256 >= ni) return; // whole workgroups past the block
  const double dt = q < ni ? start_particle(h, q) : INFINITY;
  key_min(q < ni ? order_key(ctl->desc.ti + dt) : kKeyInf, &ctl->key[ctl->phase]);
}

// Clear the step state before the first force evaluation: every particle
// due at its own (common) time, a and jerk zero as in the host driver.
__global__ __launch_bounds__(256) void hs_reset_kernel(HermiteArgs h) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h.ctl->flags = 0;
    h.ctl->done = 0;
    h.ctl->block_steps = 0;
    h.ctl->particle_steps = 0;
  }
  if (k >= h.n) return;
  const size_t cap = h.jm.cap;
  h.dt[k] = 0.0;
  for (int d = 0; d < 3; ++d) {
    h.acc[d * cap + k] = 0.0;
    h.jrk[d * cap + k] = 0.0;
    h.jm.a2[d * cap + k] = 0.0;
    h.jm.j6[d * cap + k] = 0.0;
  }
}

// ---------------------------------------------------------------- launchers

static inline dim3 grid_n(int n) { return dim3(static_cast<unsigned>((n > 0 ? n : 1) + 255) / 256); }

hipError_t launch_hs_reset(const HermiteArgs &h, hipStream_t s) {
  hipLaunchKernelGGL(hs_reset_kernel, grid_n(h.n), dim3(256), 0, s, h);
  return hipGetLastError();
}
hipError_t launch_hs_select(const HermiteArgs &h, const BatchArgs &b, hipStream_t s) {
  hipLaunchKernelGGL(hs_select_kernel, grid_n(h.n), dim3(256), 0, s, h);
  hipLaunchKernelGGL(hs_publish_kernel, dim3(1), dim3(256), 0, s, h, b);
  return hipGetLastError();
}
hipError_t launch_hs_start(const HermiteArgs &h, hipStream_t s) {
  hipLaunchKernelGGL(hs_start_kernel, grid_n(h.n), dim3(256), 0, s, h);
  return hipGetLastError();
}
hipError_t launch_hs_correct(const HermiteArgs &h, const BatchArgs &b, int grid, hipStream_t s) {
  hipLaunchKernelGGL(hs_correct_kernel, dim3(static_cast<unsigned>(reduce_grid(grid > 0 ? grid : 1))), dim3(256), 0, s, h, b);
  return hipGetLastError();
}

} // namespace g6mi
