// Host check of the batch plan's invariants (plan_shape, plan_share, plan_order,
// plan_target, plan_splits, reduce_parts) over seeded random clusters,
// tunings and grids.  Prints one line per violated invariant and the number
// of cases; exits 1 on any violation.  Built and run by
// tests/test_plan_host.py; it calls no HIP runtime function.
#include "../../paper_0902_4463_amd/csrc/g6mi_batch_common.h"

#include <cstdint>
#include <cstdio>

using namespace g6mi;

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static uint64_t next() { // splitmix64
  uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static int pick(int lo, int hi) { return lo + static_cast<int>(next() % static_cast<uint64_t>(hi - lo + 1)); }
static int logpick(int lo, int hi) { // roughly log-uniform
  int v = lo;
  const int steps = pick(0, 24);
  for (int k = 0; k < steps && v < hi; ++k) v = v * 2 > hi ? hi : v * 2;
  return pick(lo, v);
}

static int bad = 0;
#define CHECK(cond, ...)                                                                                           \
  do {                                                                                                             \
    if (!(cond)) {                                                                                                 \
      if (bad < 20) {                                                                                              \
        std::printf("violated: %s: ", #cond);                                                                      \
        std::printf(__VA_ARGS__);                                                                                  \
        std::printf("\n");                                                                                         \
      }                                                                                                            \
      ++bad;                                                                                                       \
    }                                                                                                              \
  } while (0)

static bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int main() {
  const int cases = 200000;
  for (int it = 0; it < cases; ++it) {
    BatchTune t;
    const int iws[] = {1, 2, 4, 8, 16, 32, 64, 1024};
    const int wms[] = {1, 257, 512, 1024, 1 << 30};
    t.item_work = iws[pick(0, 7)];
    t.wide_min = wms[pick(0, 4)];
    t.max_split = logpick(1, 4096);
    const int ni = pick(0, 5) == 0 ? 0 : logpick(1, 1 << 22);
    const int nj = pick(0, 5) == 0 ? 0 : logpick(1, 1 << 22);
    const int grid = logpick(1, 4096);
    const long long batch_work = 1 + static_cast<long long>(next() % (1ull << 40));

    BatchPlan pl = plan_shape(ni, nj, t);
    const int ntiles = (nj + kTile - 1) / kTile;
    CHECK(pow2(pl.ipw) && pl.ipw <= 2 * kWG, "ni=%d ipw=%d", ni, pl.ipw);
    CHECK((pl.ipw == 2 * kWG) == (ni >= t.wide_min), "ni=%d wide_min=%d ipw=%d", ni, t.wide_min, pl.ipw);
    CHECK(static_cast<long long>(pl.nib) * pl.ipw >= ni && (pl.nib == 0 || static_cast<long long>(pl.nib - 1) * pl.ipw < ni),
          "ni=%d ipw=%d nib=%d", ni, pl.ipw, pl.nib);
    CHECK(pl.per == ntiles, "nj=%d per=%d ntiles=%d", nj, pl.per, ntiles);
    CHECK(pl.ipw == 2 * kWG || pl.ipw <= kBatchMinIpw || pl.ipw <= t.item_work * 128,
          "ipw=%d item_work=%d", pl.ipw, t.item_work);

    // the share of the grid this cluster would get in a batch of batch_work
    const long long w0 = plan_work(pl);
    const long long share = (static_cast<long long>(grid) * w0 + batch_work - 1) / batch_work;
    const int ipw0 = pl.ipw;
    const bool changed = plan_share(pl, share, t);
    const int ntiles1 = ntiles;
    CHECK(pow2(pl.ipw) && pl.ipw <= ipw0, "ipw0=%d ipw=%d", ipw0, pl.ipw);
    CHECK(!changed || pl.ipw >= (ipw0 < kBatchMinIpw ? ipw0 : kBatchMinIpw), "ipw0=%d ipw=%d", ipw0, pl.ipw);
    CHECK(static_cast<long long>(pl.nib) * pl.ipw >= ni && (pl.nib == 0 || static_cast<long long>(pl.nib - 1) * pl.ipw < ni),
          "after share ni=%d ipw=%d nib=%d", ni, pl.ipw, pl.nib);
    CHECK(pl.log2ipw >= 0 && (1 << pl.log2ipw) == pl.ipw, "ipw=%d log2=%d", pl.ipw, pl.log2ipw);
    CHECK(pl.per == ntiles1, "after share nj=%d per=%d ntiles=%d", nj, pl.per, ntiles1);

    const long long target = plan_target(batch_work, grid, t);
    CHECK(target >= 1 && target <= static_cast<long long>(t.item_work) * 128, "target=%lld", target);
    plan_splits(pl, target, t);
    CHECK(pl.per >= 1 && pl.nsplit >= 1 && pl.nsplit <= t.max_split, "per=%d nsplit=%d max=%d", pl.per, pl.nsplit,
          t.max_split);
    // every tile in exactly one split, no split empty
    CHECK(static_cast<long long>(pl.per) * pl.nsplit >= ntiles1 &&
              (ntiles1 == 0 || static_cast<long long>(pl.per) * (pl.nsplit - 1) < ntiles1),
          "ntiles=%d per=%d nsplit=%d", ntiles1, pl.per, pl.nsplit);
    // every shaped cluster has a queue class; wide blocks and only they are class 1
    const int ord = plan_order(pl);
    CHECK(ord >= 0 && ord < kItemOrders && ((ord == 1) == (pl.ipw == 2 * kWG)), "ipw=%d order=%d", pl.ipw, ord);
    // the host sizes the item table by (ni / kBatchMinIpw + 1) * max_split per cluster
    CHECK(static_cast<long long>(pl.nib) * pl.nsplit <= (static_cast<long long>(ni) / kBatchMinIpw + 1) * t.max_split,
          "ni=%d nib=%d nsplit=%d", ni, pl.nib, pl.nsplit);

    const int nib = logpick(0, 1 << 20), cap = logpick(1, 128);
    const int P = reduce_parts(nib, grid, cap);
    CHECK(pow2(P) && P <= 64 && (P == 1 || P <= cap), "P=%d cap=%d", P, cap);
    CHECK(P == 1 || static_cast<long long>(nib) * P <= grid, "nib=%d P=%d grid=%d", nib, P, grid);
    CHECK(P == 64 || 2 * P > cap || static_cast<long long>(nib) * 2 * P > grid, "not maximal: nib=%d P=%d grid=%d cap=%d",
          nib, P, grid, cap);
  }
  std::printf("cases %d violations %d\n", cases, bad);
  return bad ? 1 : 0;
}
