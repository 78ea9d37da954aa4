"""g6mi_calc_device_noalloc (work buffers in the library's static per-GPU
scratch array) against g6mi_calc_device (work buffers allocated by the
handle): the same results, bit for bit, for two calls in a row, the second
with a smaller block; the neighbour lists read after each call; and the
size limit reported as an error."""

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


def _dev_inputs(torch, jm, slots, h2):
    dev = torch.device("cuda")
    ni = len(slots)
    t_slot = torch.tensor(np.asarray(slots, dtype=np.int32), device=dev)
    xi = torch.tensor(np.ascontiguousarray(jm.x[slots]), device=dev)
    vi = torch.tensor(np.ascontiguousarray(jm.v[slots]), device=dev)
    th2 = torch.full((ni,), float(h2), dtype=torch.float64, device=dev)
    return t_slot, xi, vi, th2


def _outputs(torch, ni):
    dev = torch.device("cuda")
    return [torch.full((ni, 3), np.nan, dtype=torch.float64, device=dev),
            torch.full((ni, 3), np.nan, dtype=torch.float64, device=dev),
            torch.full((ni,), np.nan, dtype=torch.float64, device=dev),
            torch.full((ni,), -7, dtype=torch.int32, device=dev),
            torch.full((ni,), np.nan, dtype=torch.float64, device=dev)]


def _lists(g6, hid, ni):
    over = g6.check(hid, g6.g6_read_neighbour_list(hid)) == g6.WARN
    counts = np.zeros(ni, dtype=np.int64)
    lists = np.full((ni, g6.NB_MAX), -1, dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    for i in range(ni):
        buf = np.zeros(g6.NB_MAX, dtype=np.int32)
        g6.check(hid, g6.g6_get_neighbour_list(hid, i, g6.NB_MAX, ln, buf))
        counts[i] = ln[0]
        k = min(int(ln[0]), g6.NB_MAX)
        lists[i, :k] = buf[:k]
    return over, counts, lists


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_noalloc_matches_calc_device(g6, prec):
    import oracle
    import torch
    jm = workloads.random_cluster(6000, seed=4242)
    eps2, h2 = 1e-4, 0.05
    hid = 7
    g6.check(hid, g6.g6_open(hid))
    try:
        g6.check(hid, g6.g6mi_set_precision(hid, prec))
        dev = torch.device("cuda")
        d = {k: torch.tensor(getattr(jm, k), device=dev) for k in ("t", "m", "index", "x", "v", "a2", "j6")}
        g6.check(hid, g6.g6mi_set_j_particles_device(hid, jm.n, d["t"], d["m"], d["index"], d["x"], d["v"],
                                                    d["a2"], d["j6"]))
        g6.g6_set_ti(hid, jm.meta["ti"])
        xp, vp = oracle.predict(jm.meta["ti"], jm.t, jm.x, jm.v, jm.a2, jm.j6)
        stream = torch.cuda.current_stream()
        # a block of several i-blocks (separate predictor), then one of a
        # single i-block (predictor fused into the interaction kernel)
        for ni in (3000, 100):
            slots = workloads.active_set(jm.n, ni, seed=ni)
            args = _dev_inputs(torch, jm, slots, h2)
            _say(f"[noalloc] {prec} ni={ni}: g6mi_calc_device")
            ref_out = _outputs(torch, ni)
            g6.check(hid, g6.g6mi_calc_device(hid, jm.n, ni, *args[:3], eps2, args[3], *ref_out, stream=stream))
            torch.cuda.synchronize()
            ref_shape = g6.g6mi_get_shape(hid)
            ref_lists = _lists(g6, hid, ni)
            _say(f"[noalloc] {prec} ni={ni}: g6mi_calc_device_noalloc")
            out = _outputs(torch, ni)
            g6.check(hid, g6.g6mi_calc_device_noalloc(hid, jm.n, ni, *args[:3], eps2, args[3], *out,
                                                      stream=stream))
            torch.cuda.synchronize()
            shape = g6.g6mi_get_shape(hid)
            lists = _lists(g6, hid, ni)
            assert shape == ref_shape, (shape, ref_shape)
            for a, b in zip(out, ref_out):
                assert torch.equal(a, b)
            assert lists[0] == ref_lists[0]
            assert np.array_equal(lists[1], ref_lists[1]) and np.array_equal(lists[2], ref_lists[2])
            # and the oracle's tolerances
            ref = oracle.force(xp, vp, jm.m, jm.index, jm.x[slots], jm.v[slots], jm.index[slots], eps2, h2,
                               conditioning=True)
            res = [o.cpu().numpy() for o in out]
            rep = parity.force_report(dict(acc=res[0], jerk=res[1], pot=res[2]), ref)
            nn = parity.nn_report(res[3], ref["nn_index"], ref["nn_r2"], xp, jm.index, jm.x[slots])
            nb = parity.nb_report(lists[1], lists[2], ref["nb_count"], ref["nb_list"], xp, jm.index, jm.x[slots],
                                  h2)
            _say(f"[noalloc] {prec} ni={ni}: shape={shape} acc_max={rep['acc_max']:.2e} nn={nn['ok']} nb={nb['ok']}")
            assert rep["ok"] and nn["ok"] and nb["ok"], (rep, nn, nb)
    finally:
        g6.g6_close(hid)


def test_noalloc_rejects_oversized_and_pending(g6):
    import torch
    hid = 8
    g6.check(hid, g6.g6_open(hid))
    try:
        dev = torch.device("cuda")
        # float64 records of 2^21 slots (128 MiB) cannot fit the scratch array
        n = 2 ** 21
        jm = workloads.make_jmemory(np.random.default_rng(5).normal(size=(n, 3)), np.zeros((n, 3)),
                                    np.full(n, 1.0 / n), meta=dict(ti=0.0))
        d = {k: torch.tensor(getattr(jm, k), device=dev) for k in ("t", "m", "index", "x", "v", "a2", "j6")}
        g6.check(hid, g6.g6mi_set_precision(hid, "fp64"))
        g6.check(hid, g6.g6mi_set_j_particles_device(hid, n, d["t"], d["m"], d["index"], d["x"], d["v"], d["a2"],
                                                    d["j6"]))
        ni = 1024
        slots = np.arange(ni)
        args = _dev_inputs(torch, jm, slots, 0.01)
        out = _outputs(torch, ni)
        _say("[noalloc] oversized call")
        assert g6.g6mi_calc_device_noalloc(hid, n, ni, *args[:3], 1e-4, args[3], *out) == g6.EINVAL
        assert "scratch" in g6.last_error(hid)
        # a j-particle set on the host and not uploaded yet
        g6.check(hid, g6.g6_set_j_particle(hid, 5, 5, 0.0, 0.0, 1.0, np.zeros(3), np.zeros(3), np.zeros(3),
                                           np.zeros(3), np.ones(3)))
        assert g6.g6mi_calc_device_noalloc(hid, n, 4, *[a[:4] for a in args[:3]], 1e-4, args[3][:4],
                                           *[o[:4] for o in out]) == g6.ESTATE
    finally:
        g6.g6_close(hid)
