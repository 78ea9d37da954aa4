"""GPU parity of the batched multi-cluster calls against the float64 oracle.

A batch holds independent clusters of uneven size, each with its own
prediction time, softening and active block.  The oracle evaluates every
cluster on its own (its j-slots predicted to its own time, its active
particles as i-particles); the batched GPU results of the cluster's rows
must meet the same tolerances as a single-system calculation.
"""

import functools
import sys

import numpy as np
import pytest

import workloads
from tests import parity

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g6():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_0902_4463_amd as g6
    return g6


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


@pytest.fixture()
def sess(g6):
    s = g6.Session(2)
    g6.check(s.id, g6.g6mi_batch_set_tuning(s.id, None))
    yield s
    s.close()


@functools.lru_cache(maxsize=4)
def small_batch(seed=41, nclusters=12, n_lo=64, n_hi=1500):
    return workloads.config_c4(seed=seed, nclusters=nclusters, n_lo=n_lo, n_hi=n_hi)


def predicted(orc, cb):
    """Every cluster's j-slots predicted to its own time (global slot order)."""
    jm = cb.jm
    xp = np.empty_like(jm.x)
    vp = np.empty_like(jm.v)
    for c in range(cb.nclusters):
        lo, hi = int(cb.joff[c]), int(cb.joff[c + 1])
        xp[lo:hi], vp[lo:hi] = orc.predict(cb.ti[c], jm.t[lo:hi], jm.x[lo:hi], jm.v[lo:hi], jm.a2[lo:hi],
                                           jm.j6[lo:hi])
    return xp, vp


def i_block(cb, xp, vp):
    """Host-predicted i-state of the active particles (the client's job)."""
    rows = cb.active
    h2 = np.repeat(cb.h2, np.diff(cb.ioff))
    return xp[rows].copy(), vp[rows].copy(), h2


def oracle_rows(orc, cb, xp, vp, xi, vi, h2, rows=None):
    """Oracle results for the given rows of the batch (all rows by default),
    each against its own cluster's j-slots."""
    jm = cb.jm
    n = len(cb.active)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    cl_of = np.searchsorted(cb.ioff, rows, side="right") - 1
    parts = []
    for c in np.unique(cl_of):
        r = rows[cl_of == c]
        lo, hi = int(cb.joff[c]), int(cb.joff[c + 1])
        ref = orc.force(xp[lo:hi], vp[lo:hi], jm.m[lo:hi], jm.index[lo:hi], xi[r], vi[r], jm.index[cb.active[r]],
                        cb.eps2[c], h2[r], conditioning=True)
        ref["_rows"] = r
        parts.append(ref)
    order = np.argsort(np.concatenate([p["_rows"] for p in parts]), kind="stable")
    out = {}
    for k in ("acc", "jerk", "pot", "acc_abs", "jerk_abs", "nn_index", "nn_r2", "nb_count", "nb_list"):
        out[k] = np.concatenate([p[k] for p in parts])[order]
    out["_rows"] = rows
    return out


def descriptors(g6, cb):
    return g6.clusters(cb.joff[:-1], np.diff(cb.joff), cb.ioff[:-1], np.diff(cb.ioff), cb.ti, cb.eps2)


class Batch:
    """Device buffers of one batch (i-arrays and outputs) and its host
    descriptors; the outputs start as NaN / -7 sentinels."""

    def __init__(self, g6, cb, xi, vi, h2, active=None, cl=None):
        import torch
        dev = torch.device("cuda")
        self.g6 = g6
        active = cb.active if active is None else active
        self.n = len(active)
        self.cl = descriptors(g6, cb) if cl is None else cl
        self.islot = torch.tensor(np.asarray(active, dtype=np.int32), device=dev)
        self.xi = torch.tensor(np.ascontiguousarray(xi), device=dev)
        self.vi = torch.tensor(np.ascontiguousarray(vi), device=dev)
        self.h2 = torch.tensor(np.ascontiguousarray(h2, dtype=np.float64), device=dev)
        n = max(self.n, 1)
        self.acc = torch.full((n, 3), float("nan"), dtype=torch.float64, device=dev)
        self.jerk = torch.full((n, 3), float("nan"), dtype=torch.float64, device=dev)
        self.pot = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        self.nnb = torch.full((n,), -7, dtype=torch.int32, device=dev)
        self.r2nn = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)

    def args(self):
        return (self.islot, self.xi, self.vi, self.h2, self.acc, self.jerk, self.pot, self.nnb, self.r2nn)

    def run(self, hid, cl=None, stream=None):
        cl = self.cl if cl is None else cl
        return self.g6.g6mi_batch_calc(hid, cl, self.n, *self.args(), stream=stream)

    def fetch(self):
        import torch
        torch.cuda.synchronize()
        n = self.n
        return dict(acc=self.acc.cpu().numpy()[:n], jerk=self.jerk.cpu().numpy()[:n], pot=self.pot.cpu().numpy()[:n],
                    nn_index=self.nnb.cpu().numpy()[:n], nn_r2=self.r2nn.cpu().numpy()[:n])


def read_lists(g6, hid, rows):
    cnt = np.zeros(len(rows), dtype=np.int64)
    lists = np.full((len(rows), 256), -1, dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    for q, r in enumerate(rows):
        buf = np.zeros(256, dtype=np.int32)
        g6.check(hid, g6.g6_get_neighbour_list(hid, int(r), 256, ln, buf))
        cnt[q] = ln[0]
        k = min(256, int(ln[0]))
        lists[q, :k] = buf[:k]
    return cnt, lists


def check_rows(g6, hid, gpu, ref, cb, xp, xi, label, strict=True, lists=True):
    rows = ref["_rows"]
    g = {k: v[rows] for k, v in gpu.items()}
    rep = parity.force_report(g, ref)
    nn = parity.nn_report(g["nn_index"], ref["nn_index"], ref["nn_r2"], xp, cb.jm.index, xi[rows])
    msg = (f"[{label}] acc_max={rep['acc_max']:.2e} jerk_max={rep['jerk_max']:.2e} pot_max={rep['pot_max']:.2e} "
           f"cond={rep['acc_conditioned']}/{rep['jerk_conditioned']} nn_mismatch={nn['mismatch']}")
    nb = dict(ok=True, fail=0)
    if lists:
        assert g6.g6_read_neighbour_list(hid) in (0, 1)
        cnt, lst = read_lists(g6, hid, rows)
        h2 = np.repeat(cb.h2, np.diff(cb.ioff))[rows]
        nb = parity.nb_report(cnt, lst, ref["nb_count"], ref["nb_list"], xp, cb.jm.index, xi[rows], h2)
        msg += f" nb_fail={nb['fail']} nb_ties={nb['ties']}"
    _say(msg)
    if strict:
        assert rep["ok"], rep
        assert nn["ok"], nn
        assert nb["ok"], nb
        same = (g["nn_index"] == ref["nn_index"]) & np.isfinite(ref["nn_r2"])
        assert np.all(np.abs(g["nn_r2"][same] - ref["nn_r2"][same]) <= 1e-5 * ref["nn_r2"][same])
    return rep


@functools.lru_cache(maxsize=4)
def small_case(seed=41):
    import oracle
    cb = small_batch(seed)
    xp, vp = predicted(oracle, cb)
    xi, vi, h2 = i_block(cb, xp, vp)
    ref = oracle_rows(oracle, cb, xp, vp, xi, vi, h2)
    return cb, xp, vp, xi, vi, h2, ref


# ----------------------------------------------------------------- parity

@pytest.mark.parametrize("prec", ["ds", "fp64", "fp32"])
def test_batch_parity(g6, sess, prec):
    """Twelve clusters (N 64..1500, their own times, active blocks of 2^k)."""
    cb, xp, vp, xi, vi, h2, ref = small_case()
    sess.load(cb.jm)
    g6.check(sess.id, g6.g6mi_set_precision(sess.id, prec))
    b = Batch(g6, cb, xi, vi, h2)
    g6.check(sess.id, b.run(sess.id))
    gpu = b.fetch()
    rep = check_rows(g6, sess.id, gpu, ref, cb, xp, xi, f"batch {prec}", strict=prec != "fp32")
    assert g6.g6mi_last_status(sess.id) & ~g6.FLAG_NB_OVERFLOW == 0
    if prec == "fp32":
        assert rep["acc_max"] < 1e-3 and rep["pot_max"] < 1e-4
    if prec == "fp64":
        assert rep["acc_max"] < 1e-12 and rep["pot_max"] < 1e-13


def test_batch_of_many_clusters(g6, sess):
    """More clusters than the plan takes in one chunk of 256 (700 small
    clusters, N 16..160): the plan entries go through memory between its
    passes, and the item and i-block tables span several chunks."""
    import oracle
    cb = small_batch(seed=47, nclusters=700, n_lo=16, n_hi=160)
    xp, vp = predicted(oracle, cb)
    xi, vi, h2 = i_block(cb, xp, vp)
    ref = oracle_rows(oracle, cb, xp, vp, xi, vi, h2)
    sess.load(cb.jm)
    g6.check(sess.id, g6.g6mi_set_precision(sess.id, "ds"))
    b = Batch(g6, cb, xi, vi, h2)
    g6.check(sess.id, b.run(sess.id))
    check_rows(g6, sess.id, b.fetch(), ref, cb, xp, xi, "700 clusters")
    assert g6.g6mi_last_status(sess.id) & ~g6.FLAG_NB_OVERFLOW == 0


TUNINGS = [dict(item_work=1, wide_min=1, wg_per_cu=1, max_split=1),
           dict(item_work=16, wide_min=100000, wg_per_cu=2, max_split=64),
           dict(item_work=2, wide_min=257, wg_per_cu=3, max_split=3),
           dict(item_work=1, wide_min=512, wg_per_cu=8, max_split=4096),
           dict(item_work=4, wide_min=2 ** 30, wg_per_cu=0, max_split=64)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "iw{item_work}-wm{wide_min}-wg{wg_per_cu}-ms{max_split}".format(**t))
def test_batch_launch_policies(g6, sess, tuning):
    """Every launch policy (items of one tile to whole clusters, wide or
    narrow blocks, 1..8 workgroups per compute unit, the narrow-only kernel
    when wide_min exceeds the batch's rows) gives oracle parity."""
    cb, xp, vp, xi, vi, h2, ref = small_case()
    sess.load(cb.jm)
    g6.check(sess.id, g6.g6mi_batch_set_tuning(sess.id, tuning))
    assert g6.g6mi_batch_get_tuning(sess.id) == tuning
    b = Batch(g6, cb, xi, vi, h2)
    g6.check(sess.id, b.run(sess.id))
    check_rows(g6, sess.id, b.fetch(), ref, cb, xp, xi, f"policy {tuning}")


def test_batch_equals_separate_calls(g6, sess):
    """A cluster's rows in a batch agree with a separate single-system call
    on that cluster alone: identical nearest neighbours and neighbour lists
    (the same float32 pair arithmetic on the same records) and forces equal
    up to summation order.  The batch may cut a small block into smaller
    i-blocks than the single call, with more lanes per i-particle, so the
    float32 partial sums differ in order: 1e-6 relative for acceleration and
    potential, 1e-5 for jerk."""
    import torch
    cb, xp, vp, xi, vi, h2, ref = small_case()
    sess.load(cb.jm)
    b = Batch(g6, cb, xi, vi, h2)
    g6.check(sess.id, b.run(sess.id))
    gpu = b.fetch()
    assert g6.g6_read_neighbour_list(sess.id) in (0, 1)
    bcnt, blst = read_lists(g6, sess.id, np.arange(b.n))
    one = g6.Session(3)
    try:
        for c in range(cb.nclusters):
            lo, hi = int(cb.joff[c]), int(cb.joff[c + 1])
            a0, a1 = int(cb.ioff[c]), int(cb.ioff[c + 1])
            if a1 == a0:
                continue
            sub = workloads.JMemory(x=cb.jm.x[lo:hi], v=cb.jm.v[lo:hi], m=cb.jm.m[lo:hi], t=cb.jm.t[lo:hi],
                                    a2=cb.jm.a2[lo:hi], j6=cb.jm.j6[lo:hi], index=cb.jm.index[lo:hi], meta={})
            one.load(sub)
            g6.g6_set_ti(one.id, cb.ti[c])
            dev = torch.device("cuda")
            islot = torch.tensor((cb.active[a0:a1] - lo).astype(np.int32), device=dev)
            n = a1 - a0
            out = [torch.empty((n, 3), dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
                   torch.empty(n, dtype=torch.float64, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                   torch.empty(n, dtype=torch.float64, device=dev)]
            g6.check(one.id, g6.g6mi_calc_device(one.id, hi - lo, n, islot, b.xi[a0:a1], b.vi[a0:a1], cb.eps2[c],
                                                 b.h2[a0:a1], *out))
            torch.cuda.synchronize()
            acc, jerk, pot, nnb, r2nn = (t.cpu().numpy() for t in out)
            for name, x, y, tol in (("acc", acc, gpu["acc"][a0:a1], 1e-6), ("jerk", jerk, gpu["jerk"][a0:a1], 1e-5)):
                err = np.linalg.norm(x - y, axis=1) / np.maximum(np.linalg.norm(x, axis=1), 1e-300)
                assert err.max() <= tol, (c, name, err.max())
            assert np.all(np.abs(pot - gpu["pot"][a0:a1]) <= 1e-6 * np.abs(pot))
            assert np.array_equal(nnb, gpu["nn_index"][a0:a1]), c
            assert np.array_equal(r2nn, gpu["nn_r2"][a0:a1]), c
            assert g6.g6_read_neighbour_list(one.id) in (0, 1)
            cnt, lst = read_lists(g6, one.id, np.arange(n))
            assert np.array_equal(cnt, bcnt[a0:a1]), c
            assert np.array_equal(lst, blst[a0:a1]), c
    finally:
        one.close()


# ------------------------------------------------------------ graph replay

def test_batch_graph_replays(g6, sess):
    """Graph mode: the first call captures, the next ones replay the graph
    with new descriptor contents (new prediction times) and new i-states.
    Eager work and synchronisations run between the replays; every replay
    matches the oracle and equals a direct launch bitwise."""
    import oracle
    import torch
    cb0 = small_batch()
    sess.load(cb0.jm)
    g6.check(sess.id, g6.g6mi_batch_use_graph(sess.id, 1))
    stream = torch.cuda.Stream()
    scratch = torch.zeros(1 << 16, device="cuda")
    for rep in range(3):
        # the same clusters at other times: a new ti per cluster
        ti = cb0.ti + (rep + 1) * 2.0 ** -9
        cb = workloads.ClusterBatch(jm=cb0.jm, joff=cb0.joff, ioff=cb0.ioff, active=cb0.active, ti=ti,
                                    eps2=cb0.eps2, h2=cb0.h2)
        xp, vp = predicted(oracle, cb)
        xi, vi, h2 = i_block(cb, xp, vp)
        ref = oracle_rows(oracle, cb, xp, vp, xi, vi, h2)
        b = Batch(g6, cb, xi, vi, h2) if rep == 0 else b
        if rep > 0:  # same buffers, new contents
            b.xi.copy_(torch.tensor(xi, device="cuda"))
            b.vi.copy_(torch.tensor(vi, device="cuda"))
            b.cl = descriptors(g6, cb)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            g6.check(sess.id, b.run(sess.id, stream=stream))
        stream.synchronize()
        gpu = b.fetch()
        check_rows(g6, sess.id, gpu, ref, cb, xp, xi, f"graph replay {rep}")
        scratch.mul_(1.5).add_(1.0)  # eager work between replays
        torch.cuda.synchronize()
        # a direct launch of the same inputs gives the same bits
        g6.check(sess.id, g6.g6mi_batch_use_graph(sess.id, 0))
        with torch.cuda.stream(stream):
            g6.check(sess.id, b.run(sess.id, stream=stream))
        stream.synchronize()
        direct = b.fetch()
        for k in gpu:
            assert np.array_equal(gpu[k], direct[k]), (rep, k)
        g6.check(sess.id, g6.g6mi_batch_use_graph(sess.id, 1))
    g6.check(sess.id, g6.g6mi_batch_use_graph(sess.id, 0))


# ----------------------------------------------- descriptors on the device

def test_batch_device_descriptors_skip_bad_cluster(g6, sess):
    """Descriptors read from device memory: a descriptor reaching past the
    j-memory is skipped and flagged; its rows are left untouched, every
    other cluster is still correct."""
    import torch
    cb, xp, vp, xi, vi, h2, ref = small_case()
    sess.load(cb.jm)
    b = Batch(g6, cb, xi, vi, h2)
    cl = b.cl.copy()
    bad = int(np.argmax(np.diff(cb.ioff)))  # a cluster with active rows
    cl["nj"][bad] = cb.jm.n + 5
    d_cl = torch.tensor(cl.view(np.uint8), device="cuda")
    g6.check(sess.id, g6.g6mi_batch_calc_device(sess.id, len(cl), d_cl, b.n, *b.args()))
    gpu = b.fetch()
    assert g6.g6mi_last_status(sess.id) & g6.FLAG_BAD_CLUSTER
    a0, a1 = int(cb.ioff[bad]), int(cb.ioff[bad + 1])
    assert np.all(np.isnan(gpu["acc"][a0:a1])) and np.all(gpu["nn_index"][a0:a1] == -7)
    keep = np.ones(b.n, dtype=bool)
    keep[a0:a1] = False
    sub = {k: v[keep] if k != "_rows" else np.arange(keep.sum()) for k, v in ref.items()}
    g = {k: v[keep] for k, v in gpu.items()}
    rep = parity.force_report(g, sub)
    assert rep["ok"], rep
    # the host-descriptor call rejects the same descriptor before any work
    assert g6.g6mi_batch_calc(sess.id, cl, b.n, *b.args()) == g6.EINVAL
    assert "cluster" in g6.last_error(sess.id)


# ------------------------------------------------------------- edge cases

def test_batch_edge_cases(g6, sess):
    """Empty batch; clusters without i-particles; a cluster without
    j-slots (zero force, no neighbour); a one-particle cluster (its own slot
    excluded); ragged tails of one record past full tiles."""
    import oracle
    import torch
    jm = workloads.random_cluster(1100, seed=9)
    sess.load(jm)
    dev = torch.device("cuda")
    # empty batch
    z = torch.zeros(1, device=dev)
    g6.check(sess.id, g6.g6mi_batch_calc(sess.id, g6.clusters([], [], [], [], [], []), 0, z, z, z, z, z, z, z))
    torch.cuda.synchronize()
    # clusters: (joff, nj, active slots)
    spec = [(0, 257, [0, 5, 256]), (257, 0, []), (257, 1, [257]), (258, 0, []), (300, 800, list(range(300, 1100, 3)))]
    xp, vp = oracle.predict(0.0, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    active = np.array([s for _, _, a in spec for s in a], dtype=np.int64)
    counts = [len(a) for _, _, a in spec]
    ioff = np.concatenate([[0], np.cumsum(counts)])
    # i-particle 1 of the cluster without j-slots: row with a foreign particle
    xi, vi = xp[active].copy(), vp[active].copy()
    cl = g6.clusters([s[0] for s in spec], [s[1] for s in spec], ioff[:-1], counts, [0.0] * len(spec),
                     [1e-4] * len(spec))
    # a cluster with nj = 0 but one i-particle (slot 5's particle)
    cl = np.concatenate([cl, g6.clusters([600], [0], [len(active)], [1], [0.0], [1e-4])])
    active = np.concatenate([active, [5]])
    xi = np.concatenate([xi, xp[[5]]])
    vi = np.concatenate([vi, vp[[5]]])
    n = len(active)
    h2 = np.full(n, 0.05)
    b = Batch(g6, None, xi, vi, h2, active=active, cl=cl)
    g6.check(sess.id, b.run(sess.id, cl=cl))
    gpu = b.fetch()
    assert g6.g6_read_neighbour_list(sess.id) in (0, 1)
    row = 0
    for c, (joff, nj, act) in enumerate(spec):
        for s in act:
            lo, hi = joff, joff + nj
            ref = oracle.force(xp[lo:hi], vp[lo:hi], jm.m[lo:hi], jm.index[lo:hi], xi[[row]], vi[[row]],
                               jm.index[[s]], 1e-4, 0.05, conditioning=True)
            g = {k: gpu[k][[row]] for k in ("acc", "jerk", "pot")}
            if nj <= 1:  # nothing but itself: exactly zero, no neighbour
                assert np.all(g["acc"] == 0) and np.all(g["pot"] == 0) and gpu["nn_index"][row] == -1
                assert np.isinf(gpu["nn_r2"][row])
            else:
                rep = parity.force_report(g, ref)
                assert rep["ok"], (c, s, rep)
                assert gpu["nn_index"][row] == ref["nn_index"][0]
            row += 1
    # the cluster without j-slots and a foreign i-particle
    assert np.all(gpu["acc"][row] == 0) and gpu["pot"][row] == 0 and gpu["nn_index"][row] == -1
    ln = np.zeros(1, dtype=np.int32)
    buf = np.zeros(256, dtype=np.int32)
    g6.check(sess.id, g6.g6_get_neighbour_list(sess.id, row, 256, ln, buf))
    assert ln[0] == 0


def test_batch_neighbour_overflow(g6, sess):
    """A cluster whose lists overflow: the kept lists are the 256 smallest
    particle indices, exactly as the oracle's (the exact pass predicts the
    cluster's records again at the cluster's own time)."""
    import oracle
    cb = small_batch(seed=43, nclusters=4, n_lo=600, n_hi=900)
    sess.load(cb.jm)
    big = cb.h2.copy()
    big[1] = 1e6  # every particle of cluster 1 is a neighbour
    cb = workloads.ClusterBatch(jm=cb.jm, joff=cb.joff, ioff=cb.ioff, active=cb.active, ti=cb.ti, eps2=cb.eps2,
                                h2=big)
    xp, vp = predicted(oracle, cb)
    xi, vi, h2 = i_block(cb, xp, vp)
    ref = oracle_rows(oracle, cb, xp, vp, xi, vi, h2)
    b = Batch(g6, cb, xi, vi, h2)
    g6.check(sess.id, b.run(sess.id))
    b.fetch()
    a0, a1 = int(cb.ioff[1]), int(cb.ioff[2])
    assert a1 > a0
    assert g6.g6mi_last_status(sess.id) & g6.FLAG_NB_OVERFLOW
    assert g6.g6_read_neighbour_list(sess.id) == g6.WARN
    cnt, lst = read_lists(g6, sess.id, np.arange(b.n))
    assert np.array_equal(cnt, ref["nb_count"])
    over = cnt > 256
    assert over[a0:a1].all() and not over[:a0].any() and not over[a1:].any()
    assert np.array_equal(lst[over], ref["nb_list"][over])


# ------------------------------------------------------------ autotuner

def test_batch_autotune_and_cache(g6, sess, tmp_path):
    """The autotuner times the candidate policies, applies and appends the
    fastest to the cache file; a hand-written entry for another batch's key
    is applied from the file without timing; results stay correct."""
    cb, xp, vp, xi, vi, h2, ref = small_case()
    sess.load(cb.jm)
    b = Batch(g6, cb, xi, vi, h2)
    path = tmp_path / "tune.txt"
    rc, best = g6.g6mi_batch_autotune(sess.id, b.cl, b.n, *b.args(), cache_path=str(path), reps=2)
    assert rc == g6.OK, g6.last_error(sess.id)
    assert g6.g6mi_batch_get_tuning(sess.id) == best
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("g6mi-batch-tune-v2 ")
    _say(f"[autotune] {lines[0]}")
    g6.check(sess.id, b.run(sess.id))
    check_rows(g6, sess.id, b.fetch(), ref, cb, xp, xi, "autotuned", lists=False)
    # the same batch again: taken from the table, the file is unchanged
    rc, again = g6.g6mi_batch_autotune(sess.id, b.cl, b.n, *b.args(), cache_path=str(path))
    assert rc == g6.OK and again == best and len(path.read_text().splitlines()) == 1
    # another batch (fewer clusters: another key) with a hand-written entry
    cl2 = b.cl[:5]
    n2 = int(cl2["ioff"][-1] + cl2["ni"][-1])
    key = lines[0].split()[1].replace("/c12/", "/c5/")
    pair = float(np.sum(cl2["ni"].astype(float) * cl2["nj"]))
    parts = key.split("/")
    parts[-3] = f"lp{int(np.floor(np.log2(pair)))}"
    parts[-2] = f"li{int(np.floor(np.log2(max(1, n2))))}"
    parts[-1] = f"lj{int(np.floor(np.log2(float(np.sum(cl2['nj'])))))}"
    key = "/".join(parts)
    with open(path, "a") as f:
        f.write(f"g6mi-batch-tune-v2 {key} 3 300 1 7 0.5\n")
    rc, got = g6.g6mi_batch_autotune(sess.id, cl2, n2, *b.args(), cache_path=str(path))
    assert rc == g6.OK
    assert got == dict(item_work=3, wide_min=300, wg_per_cu=1, max_split=7), (got, key)


# ------------------------------------------- the batched workload, full size

@functools.lru_cache(maxsize=1)
def c4_case():
    return workloads.config_c4()


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_config_c4_full_size_sampled(g6, sess, prec):
    """256 Plummer clusters, N log-uniform in [256, 8192] (672,907 particles),
    Salpeter masses, own centres, times and active blocks (52,631 i); one
    batched launch, up to 16 rows per cluster checked against the oracle."""
    import oracle
    import torch
    cb = c4_case()
    _say(f"[C4] loading {cb.jm.n} particles in {cb.nclusters} clusters ({prec})")
    jm = cb.jm
    dev = torch.device("cuda")
    d = dict(t=torch.tensor(jm.t, device=dev), m=torch.tensor(jm.m, device=dev),
             index=torch.tensor(jm.index, device=dev), x=torch.tensor(jm.x, device=dev),
             v=torch.tensor(jm.v, device=dev), a2=torch.tensor(jm.a2, device=dev),
             j6=torch.tensor(jm.j6, device=dev))
    g6.check(sess.id, g6.g6mi_set_j_particles_device(sess.id, jm.n, d["t"], d["m"], d["index"], d["x"], d["v"],
                                                    d["a2"], d["j6"]))
    g6.check(sess.id, g6.g6mi_set_precision(sess.id, prec))
    xp, vp = predicted(oracle, cb)
    xi, vi, h2 = i_block(cb, xp, vp)
    b = Batch(g6, cb, xi, vi, h2)
    _say(f"[C4] running ({prec})")
    g6.check(sess.id, b.run(sess.id))
    gpu = b.fetch()
    rng = np.random.default_rng(4)
    rows = np.concatenate([rng.permutation(np.arange(cb.ioff[c], cb.ioff[c + 1]))[:16]
                           for c in range(cb.nclusters)]).astype(np.int64)
    rows.sort()
    ref = oracle_rows(oracle, cb, xp, vp, xi, vi, h2, rows)
    check_rows(g6, sess.id, gpu, ref, cb, xp, xi, f"C4 {prec}")
    assert np.all(np.isfinite(gpu["acc"])) and np.all(gpu["nn_index"] >= 0)
