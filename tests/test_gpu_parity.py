"""GPU parity: libg6mi (through its C ABI) against the float64 CPU oracle.

Every GPU result is compared element by element with the oracle on the same
seeded inputs.  The i-block handed to the GPU is the host-predicted state of
the active particles (the client's job in the paper's CPU/GPU split); the
j-memory is predicted independently on each side.
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
    s = g6.Session(1)
    yield s
    s.close()


def oracle_eval(orc, jm, slots, eps2, h2):
    return orc.evaluate(jm, jm.meta.get("ti", 0.0), slots, eps2, h2, conditioning=True)


def gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec, shape=(0, 0), neighbours=True):
    g6.check(sess.id, g6.g6mi_set_precision(sess.id, prec))
    g6.check(sess.id, g6.g6mi_set_shape(sess.id, *shape))
    return sess.calc(jm.n, jm.meta.get("ti", 0.0), jm.index[slots], ref["xi"], ref["vi"], eps2, h2,
                     neighbours=neighbours)


def assert_parity(gpu, ref, jm, h2, prec, label, strict=True):
    xp, _ = ref["_xp"], None
    rep = parity.force_report(gpu, ref)
    nn = parity.nn_report(gpu["nn_index"], ref["nn_index"], ref["nn_r2"], xp, jm.index, ref["xi"])
    _say(f"[{label}] {prec}: acc_max={rep['acc_max']:.2e} jerk_max={rep['jerk_max']:.2e} "
         f"pot_max={rep['pot_max']:.2e} cond={rep['acc_conditioned']}/{rep['jerk_conditioned']} "
         f"nn_mismatch={nn['mismatch']} nn_ties={nn['ties']}")
    if "nb_count" in gpu:
        nb = parity.nb_report(gpu["nb_count"], gpu["nb_list"], ref["nb_count"], ref["nb_list"], xp, jm.index,
                              ref["xi"], h2)
        _say(f"[{label}] {prec}: nb_fail={nb['fail']} nb_ties={nb['ties']}")
    else:
        nb = dict(ok=True)
    if strict:
        assert rep["ok"], rep
        assert nn["ok"], nn
        assert nb["ok"], nb
        # r2 of the nearest neighbour, where the index agrees
        same = gpu["nn_index"] == ref["nn_index"]
        fin = same & np.isfinite(ref["nn_r2"])
        assert np.all(np.abs(gpu["nn_r2"][fin] - ref["nn_r2"][fin]) <= 1e-5 * ref["nn_r2"][fin])
    return rep


def with_xp(orc, jm, ref):
    xp, _ = orc.predict(jm.meta.get("ti", 0.0), jm.t, jm.x, jm.v, jm.a2, jm.j6)
    ref["_xp"] = xp
    return ref


# ------------------------------------------------------------------ C1

@pytest.mark.parametrize("prec", ["ds", "fp64", "fp32"])
def test_config_c1_full_evaluation(g6, orc, sess, prec):
    """Equal-mass Plummer N=1024, eps = 1/64, all particles active."""
    jm = workloads.config_c1()
    slots = np.arange(jm.n)
    eps2, h2 = jm.meta["eps2"], jm.meta["h2"]
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    gpu = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec)
    rep = assert_parity(gpu, ref, jm, h2, prec, "C1", strict=prec != "fp32")
    if prec == "fp32":
        assert rep["acc_max"] < 1e-4 and rep["pot_max"] < 1e-5
    if prec == "fp64":
        assert rep["acc_max"] < 1e-12 and rep["jerk_max"] < 1e-11 and rep["pot_max"] < 1e-13
    # Newton's third law on the GPU output, to the force tolerance
    tot = (jm.m[:, None] * gpu["acc"]).sum(axis=0)
    assert np.all(np.abs(tot) <= 2e-6 * np.sum(jm.m * np.linalg.norm(gpu["acc"], axis=1)))


# --------------------------------------------- sizes spanning tiles and tails

CASES = [(1, 1), (2, 1), (3, 3), (63, 7), (64, 64), (65, 7), (255, 64), (256, 256), (257, 257),
         (4097, 300), (4097, 1), (5000, 7)]


@pytest.mark.parametrize("n,ni", CASES)
@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_sizes_and_tails(g6, orc, sess, n, ni, prec):
    jm = workloads.random_cluster(n, seed=1000 + n)
    slots = workloads.active_set(n, ni, seed=n)
    eps2, h2 = 1e-4, 0.05
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    gpu = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec)
    assert_parity(gpu, ref, jm, h2, prec, f"N={n} ni={ni}")


@pytest.mark.parametrize("prec", ["ds", "fp64"])
@pytest.mark.parametrize("ni,shape", [(300, (0, 0)), (40, (0, 0)), (1500, (512, 3)), (300, (64, 5))])
def test_self_tiles_unsoftened(g6, orc, sess, prec, ni, shape):
    """A random subset of the particles as the block, so that nearly every
    full tile holds some lane's own slot (the grouped path with the own pair
    left out per pair), without softening: the own pair would add an
    infinite term, or be its own nearest neighbour and neighbour, if it were
    not left out exactly."""
    n = 4096
    jm = workloads.random_cluster(n, seed=77)
    slots = workloads.active_set(n, ni, seed=78)
    eps2, h2 = 0.0, 0.05
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    gpu = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec, shape=shape)
    assert np.all(np.isfinite(gpu["acc"])) and np.all(np.isfinite(gpu["jerk"])) and np.all(np.isfinite(gpu["pot"]))
    assert np.all(gpu["nn_index"] != jm.index[slots])
    assert_parity(gpu, ref, jm, h2, prec, f"self tiles eps=0 ni={ni} shape={shape}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (4, 3), (64, 7), (256, 1), (8, 100), (2, 13), (128, 2),
                                   (512, 1), (512, 5)])
def test_launch_shapes(g6, orc, sess, shape):
    """Every (i per workgroup, j-split) choice gives results within
    tolerance, and the same shape twice gives identical bits."""
    jm = workloads.random_cluster(3001, seed=77)
    slots = workloads.active_set(3001, 700, seed=5)
    eps2, h2 = 1e-3, 0.03
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    a = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds", shape)
    used = g6.g6mi_get_shape(sess.id)
    assert used["i_per_group"] == shape[0] and used["j_splits"] == min(shape[1], (3001 + 255) // 256)
    assert_parity(a, ref, jm, h2, "ds", f"shape={shape}")
    b = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds", shape)
    for key in ("acc", "jerk", "pot", "nn_index", "nn_r2", "nb_count", "nb_list"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("prec", ["ds", "fp64"])
@pytest.mark.parametrize("shape", [(1, 79), (4, 37), (16, 64), (256, 9), (32, 17)])
def test_split_sums_over_lane_groups(g6, orc, sess, prec, shape):
    """Many j-splits of few i-particles: the reduction adds each
    i-particle's splits over a group of lanes (4..64 lanes, ragged split
    counts per lane) and still meets the tolerance, with identical bits on a
    repeated call and the same nearest neighbours as the oracle."""
    jm = workloads.random_cluster(20000, seed=81)
    slots = workloads.active_set(20000, 45, seed=6)
    eps2, h2 = 1e-4, 0.01
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    a = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec, shape)
    assert g6.g6mi_get_shape(sess.id)["j_splits"] == shape[1]
    assert_parity(a, ref, jm, h2, prec, f"splits shape={shape}")
    b = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec, shape)
    for key in ("acc", "jerk", "pot", "nn_index", "nn_r2", "nb_count", "nb_list"):
        assert np.array_equal(a[key], b[key]), key


def test_i_particles_outside_jmemory(g6, orc, sess):
    """i-particles whose index is not stored in the j-memory feel every
    j-particle (no self exclusion)."""
    jm = workloads.random_cluster(700, seed=3)
    rng = np.random.default_rng(4)
    xi = rng.normal(size=(50, 3)) * 0.5
    vi = rng.normal(size=(50, 3)) * 0.5
    idx = np.arange(10 ** 6, 10 ** 6 + 50, dtype=np.int32)
    xp, vp = orc.predict(jm.meta["ti"], jm.t, jm.x, jm.v, jm.a2, jm.j6)
    ref = orc.force(xp, vp, jm.m, jm.index, xi, vi, idx, 1e-4, 0.05, conditioning=True)
    ref["xi"], ref["vi"], ref["_xp"] = xi, vi, xp
    sess.load(jm)
    g6.g6mi_set_precision(sess.id, "ds")
    g6.g6mi_set_shape(sess.id, 0, 0)
    gpu = sess.calc(jm.n, jm.meta["ti"], idx, xi, vi, 1e-4, 0.05)
    assert_parity(gpu, ref, jm, 0.05, "ds", "foreign i")


# ------------------------------------------------------------- edge cases

def test_neighbour_overflow(g6, orc, sess):
    rng = np.random.default_rng(61)
    n = 700
    x = rng.normal(size=(n, 3)) * 0.01
    jm = workloads.make_jmemory(x, rng.normal(size=(n, 3)), np.full(n, 1 / n), meta=dict(ti=0.0))
    slots = np.arange(0, n, 50)
    ref = oracle_eval(orc, jm, slots, 1e-6, 1.0)
    sess.load(jm)
    g6.g6mi_set_precision(sess.id, "ds")
    g6.g6mi_set_shape(sess.id, 0, 0)
    gpu = sess.calc(n, 0.0, jm.index[slots], ref["xi"], ref["vi"], 1e-6, 1.0)
    assert gpu["nb_overflow"]
    assert np.array_equal(gpu["nb_count"], ref["nb_count"])
    # the kept entries are the 256 smallest indices, as in the oracle
    assert np.array_equal(gpu["nb_list"], ref["nb_list"])


@pytest.mark.parametrize("prec", ["ds", "fp64", "fp32"])
def test_neighbour_overflow_shuffled_indices(g6, orc, sess, prec):
    """Overflowing lists with particle indices unrelated to slots, some
    negative: the exact pass keeps the 256 smallest indices; rows that do not
    overflow are untouched."""
    rng = np.random.default_rng(62)
    n = 3000
    x = rng.normal(size=(n, 3)) * 0.05
    idx = rng.permutation(np.arange(-1500, n - 1500)).astype(np.int32)
    jm = workloads.make_jmemory(x, rng.normal(size=(n, 3)), np.full(n, 1 / n), index=idx, meta=dict(ti=0.0))
    slots = np.arange(0, n, 7)
    h2 = np.where(np.arange(len(slots)) % 2 == 0, 0.02, 1e-4)
    ref = oracle_eval(orc, jm, slots, 1e-6, h2)
    sess.load(jm)
    g6.g6mi_set_precision(sess.id, prec)
    g6.g6mi_set_shape(sess.id, 0, 0)
    gpu = sess.calc(n, 0.0, jm.index[slots], ref["xi"], ref["vi"], 1e-6, h2)
    assert gpu["nb_overflow"] and (ref["nb_count"] > 256).any() and (ref["nb_count"] <= 256).any()
    xp, _ = orc.predict(0.0, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    nb = parity.nb_report(gpu["nb_count"], gpu["nb_list"], ref["nb_count"], ref["nb_list"], xp, jm.index,
                          ref["xi"], h2)
    over = ref["nb_count"] > 256
    # counts may differ only through ties at the radius; overflowing rows are exact
    same = gpu["nb_count"] == ref["nb_count"]
    assert same.mean() > 0.95
    for r in np.nonzero(over & same)[0]:
        assert np.array_equal(gpu["nb_list"][r], ref["nb_list"][r]), r
    assert nb["ok"], nb


# ------------------------------------------- predictor fused into small blocks

FUSED_CASES = [(1, 1), (4097, 1), (4097, 7), (5000, 256), (700, 100), (300, 256)]


@pytest.mark.parametrize("n,ni", FUSED_CASES)
@pytest.mark.parametrize("prec", ["ds", "fp64", "fp32"])
def test_fused_prediction_matches_separate_predictor(g6, orc, sess, n, ni, prec):
    """Blocks of at most 256 i-particles predict their j-tiles inside the
    interaction kernel, with the arithmetic of the separate predictor: the
    results agree with that path bit for bit and meet the oracle's
    tolerances (float32 reported, not graded)."""
    jm = workloads.random_cluster(n, seed=3000 + n)
    slots = workloads.active_set(n, ni, seed=ni)
    eps2, h2 = 1e-4, 0.05
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    fused = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec)
    g6.check(sess.id, g6.g6mi_set_fused_predict(sess.id, 0))
    try:
        sep = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec)
    finally:
        g6.check(sess.id, g6.g6mi_set_fused_predict(sess.id, 1))
    for key in ("acc", "jerk", "pot", "nn_index", "nn_r2", "nb_count", "nb_list"):
        assert np.array_equal(fused[key], sep[key]), key
    assert_parity(fused, ref, jm, h2, prec, f"fused N={n} ni={ni}", strict=prec != "fp32")


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_fused_neighbour_overflow_and_fresh_counters(g6, orc, sess, prec):
    """Fused small blocks in a row on one handle: lists that all overflow
    (the exact pass predicts the records again from the j-memory), a call
    with lists near their radius, and again overflowing lists: each call
    starts from cleared counters, which no launch clears beforehand (the
    reduction of the previous call does)."""
    rng = np.random.default_rng(63)
    n = 3000
    x = rng.normal(size=(n, 3)) * 0.01
    idx = (rng.permutation(n) * 3 + 5).astype(np.int32)
    jm = workloads.make_jmemory(x, rng.normal(size=(n, 3)), np.full(n, 1 / n), index=idx, meta=dict(ti=0.0))
    sess.load(jm)
    xp, _ = orc.predict(0.0, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    for ni, h2 in ((200, 1.0), (37, 1e-5), (5, 1.0), (200, 1e-5)):
        slots = workloads.active_set(n, ni, seed=ni)
        ref = oracle_eval(orc, jm, slots, 1e-6, h2)
        gpu = gpu_eval(sess, g6, jm, slots, ref, 1e-6, h2, prec)
        if h2 == 1.0:
            assert gpu["nb_overflow"] and (ref["nb_count"] > 256).all()
            assert np.array_equal(gpu["nb_count"], ref["nb_count"])
            assert np.array_equal(gpu["nb_list"], ref["nb_list"])
        else:
            nb = parity.nb_report(gpu["nb_count"], gpu["nb_list"], ref["nb_count"], ref["nb_list"], xp, jm.index,
                                  ref["xi"], h2)
            assert nb["ok"] and nb["overflow_rows"] == 0, nb


def test_nonfinite_output_is_flagged(g6, sess):
    """eps = 0 with two distinct particles at the same place: the result is
    not finite and lasthalf says so with return code 1."""
    x = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    jm = workloads.make_jmemory(x, np.zeros((3, 3)), np.ones(3), meta=dict(ti=0.0))
    sess.load(jm)
    g6.g6mi_set_precision(sess.id, "ds")
    ni = 1
    g6.g6_set_ti(sess.id, 0.0)
    assert g6.g6calc_firsthalf(sess.id, 3, ni, [0], x[:1], np.zeros((1, 3)), None, None, None, 0.0, [0.1]) == 0
    acc = np.zeros((1, 3)); jerk = np.zeros((1, 3)); pot = np.zeros(1)
    assert g6.g6calc_lasthalf(sess.id, 3, ni, [0], x[:1], np.zeros((1, 3)), 0.0, [0.1], acc, jerk, pot) == g6.WARN


def test_empty_j_and_empty_i(g6, sess):
    jm = workloads.random_cluster(10, seed=9)
    sess.load(jm)
    g6.g6mi_set_precision(sess.id, "ds")
    out = sess.calc(0, 0.0, np.array([3, 4], dtype=np.int32), jm.x[3:5], jm.v[3:5], 1e-4, 0.1)
    assert np.all(out["acc"] == 0) and np.all(out["pot"] == 0) and np.all(out["jerk"] == 0)
    assert np.all(out["nn_index"] == -1) and np.all(np.isinf(out["nn_r2"]))
    assert np.all(out["nb_count"] == 0)
    out = sess.calc(10, 0.0, np.zeros(0, dtype=np.int32), np.zeros((0, 3)), np.zeros((0, 3)), 1e-4, 0.1)
    assert out["acc"].shape == (0, 3)


def test_call_sequence_errors(g6, sess):
    jm = workloads.random_cluster(20, seed=2)
    sess.load(jm)
    acc = np.zeros((2, 3)); jerk = np.zeros((2, 3)); pot = np.zeros(2)
    idx = np.array([0, 1], dtype=np.int32)
    assert g6.g6calc_lasthalf(sess.id, 20, 2, idx, None, None, 1e-4, None, acc, jerk, pot) == g6.ESTATE
    assert g6.g6calc_firsthalf(sess.id, 21, 2, idx, jm.x[:2], jm.v[:2], None, None, None, 1e-4, None) == g6.EINVAL
    assert g6.g6calc_lasthalf(sess.id, 21, 2, idx, None, None, 1e-4, None, acc, jerk, pot) == g6.EINVAL
    assert g6.g6calc_firsthalf(sess.id, 20, 2, idx, jm.x[:2], jm.v[:2], None, None, None, 1e-4, None) == 0
    assert g6.g6calc_lasthalf(sess.id, 20, 2, idx, None, None, 2e-4, None, acc, jerk, pot) == g6.EINVAL
    assert g6.g6calc_firsthalf(sess.id, 20, 2, idx, jm.x[:2], jm.v[:2], None, None, None, -1.0, None) == g6.EINVAL
    assert g6.g6calc_lasthalf(sess.id, 20, 2, idx, None, None, -1.0, None, acc, jerk, pot) == g6.EINVAL
    bad = jm.x[:2].copy(); bad[0, 0] = np.nan
    assert g6.g6calc_firsthalf(sess.id, 20, 2, idx, bad, jm.v[:2], None, None, None, 1e-4, None) == g6.EINVAL
    assert g6.g6calc_lasthalf(sess.id, 20, 2, idx, None, None, 1e-4, None, acc, jerk, pot) == g6.EINVAL
    assert g6.g6mi_set_shape(sess.id, 3, 1) == g6.EINVAL
    assert g6.g6mi_set_precision(sess.id, 7) == g6.EINVAL


def test_neighbour_lists_switch(g6, orc, sess):
    """Turning neighbour lists off leaves forces bit-identical and reports
    empty lists."""
    jm = workloads.random_cluster(2000, seed=12)
    slots = workloads.active_set(2000, 200, seed=1)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 1e-4, 0.05))
    sess.load(jm)
    on = gpu_eval(sess, g6, jm, slots, ref, 1e-4, 0.05, "ds")
    g6.g6mi_set_neighbour_lists(sess.id, 0)
    off = gpu_eval(sess, g6, jm, slots, ref, 1e-4, 0.05, "ds")
    g6.g6mi_set_neighbour_lists(sess.id, 1)
    for key in ("acc", "jerk", "pot", "nn_index"):
        assert np.array_equal(on[key], off[key])
    assert np.all(off["nb_count"] == 0)


def test_set_j_particle_updates_between_calls(g6, orc, sess):
    """Re-storing some j-particles (a corrector step) changes only what the
    next calculation sees: results match the oracle on the updated memory."""
    jm = workloads.random_cluster(1500, seed=14)
    sess.load(jm)
    rng = np.random.default_rng(2)
    upd = rng.choice(1500, 100, replace=False)
    jm.x[upd] += rng.normal(size=(100, 3)) * 0.01
    jm.t[upd] = jm.meta["ti"]
    zero = np.zeros(3)
    for k in upd:
        g6.check(sess.id, g6.g6_set_j_particle(sess.id, int(k), int(jm.index[k]), jm.t[k], 0.0, jm.m[k], zero,
                                              jm.j6[k], jm.a2[k], jm.v[k], jm.x[k]))
    slots = workloads.active_set(1500, 128, seed=3)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 1e-4, 0.05))
    gpu = gpu_eval(sess, g6, jm, slots, ref, 1e-4, 0.05, "ds")
    assert_parity(gpu, ref, jm, 0.05, "ds", "updated j")


# ---------------------------------------------------- device-resident path

def device_jmem(g6, sess, jm):
    import torch
    dev = torch.device("cuda")
    d = dict(t=torch.tensor(jm.t, device=dev), m=torch.tensor(jm.m, device=dev),
             index=torch.tensor(jm.index, device=dev), x=torch.tensor(jm.x, device=dev),
             v=torch.tensor(jm.v, device=dev), a2=torch.tensor(jm.a2, device=dev),
             j6=torch.tensor(jm.j6, device=dev))
    g6.check(sess.id, g6.g6mi_set_j_particles_device(sess.id, jm.n, d["t"], d["m"], d["index"], d["x"], d["v"],
                                                    d["a2"], d["j6"]))
    torch.cuda.synchronize()
    return d


def device_calc(g6, sess, nj, islot, xi, vi, eps2, h2):
    import torch
    dev = torch.device("cuda")
    ni = len(islot)
    t_islot = torch.tensor(np.asarray(islot, dtype=np.int32), device=dev)
    t_xi = torch.tensor(np.ascontiguousarray(xi), device=dev)
    t_vi = torch.tensor(np.ascontiguousarray(vi), device=dev)
    t_h2 = torch.tensor(np.broadcast_to(np.float64(h2), (ni,)).copy(), device=dev)
    out = dict(acc=torch.empty((ni, 3), dtype=torch.float64, device=dev),
               jerk=torch.empty((ni, 3), dtype=torch.float64, device=dev),
               pot=torch.empty(ni, dtype=torch.float64, device=dev),
               nnb=torch.empty(ni, dtype=torch.int32, device=dev),
               r2nn=torch.empty(ni, dtype=torch.float64, device=dev))
    stream = torch.cuda.current_stream()
    g6.check(sess.id, g6.g6mi_calc_device(sess.id, nj, ni, t_islot, t_xi, t_vi, eps2, t_h2, out["acc"],
                                          out["jerk"], out["pot"], out["nnb"], out["r2nn"], stream=stream))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_device_path_matches_host_path(g6, orc, sess):
    jm = workloads.random_cluster(3000, seed=17)
    slots = workloads.active_set(3000, 333, seed=2)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 1e-4, 0.05))
    sess.load(jm)
    host = gpu_eval(sess, g6, jm, slots, ref, 1e-4, 0.05, "ds")
    device_jmem(g6, sess, jm)
    g6.g6_set_ti(sess.id, jm.meta["ti"])
    dv = device_calc(g6, sess, jm.n, slots, ref["xi"], ref["vi"], 1e-4, 0.05)
    for k_host, k_dev in (("acc", "acc"), ("jerk", "jerk"), ("pot", "pot"), ("nn_index", "nnb"), ("nn_r2", "r2nn")):
        assert np.array_equal(host[k_host], dv[k_dev]), k_host


# --------------------------------------- full-size workloads, sampled outputs

@functools.lru_cache(maxsize=1)
def c3_case(n=2 ** 20):
    return workloads.config_c3(n=n)


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_config_c3_full_size_sampled(g6, orc, sess, prec):
    """Plummer N=2^20 with Salpeter masses: all 2^20 particles active (the
    benchmark's launch), 512 sampled i-particles checked against the
    oracle.  The i-block is the stored (unpredicted) state, as in the
    benchmark; both sides get the same arrays."""
    import torch
    jm = c3_case()
    n = jm.n
    eps2, h2, ti = jm.meta["eps2"], jm.meta["h2"], jm.meta["ti"]
    _say(f"[C3] loading N={n} ({prec})")
    device_jmem(g6, sess, jm)
    g6.g6mi_set_precision(sess.id, prec)
    g6.g6mi_set_shape(sess.id, 0, 0)
    g6.g6_set_ti(sess.id, ti)
    slots = np.arange(n, dtype=np.int32)
    _say(f"[C3] running ni={n} ({prec})")
    dv = device_calc(g6, sess, n, slots, jm.x, jm.v, eps2, h2)
    sample = workloads.active_set(n, 512, seed=33)
    xp, vp = orc.predict(ti, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    ref = orc.force(xp, vp, jm.m, jm.index, jm.x[sample], jm.v[sample], jm.index[sample], eps2, h2,
                    conditioning=True)
    gpu = dict(acc=dv["acc"][sample], jerk=dv["jerk"][sample], pot=dv["pot"][sample])
    rep = parity.force_report(gpu, ref)
    nn = parity.nn_report(dv["nnb"][sample], ref["nn_index"], ref["nn_r2"], xp, jm.index, jm.x[sample])
    _say(f"[C3] {prec}: {rep} nn={nn}")
    assert rep["ok"], rep
    assert nn["ok"], nn
    # neighbour lists of the sampled particles
    assert g6.g6_read_neighbour_list(sess.id) in (0, 1)
    cnt = np.zeros(len(sample), dtype=np.int64)
    lists = np.full((len(sample), 256), -1, dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    for q, i in enumerate(sample):
        buf = np.zeros(256, dtype=np.int32)
        g6.g6_get_neighbour_list(sess.id, int(i), 256, ln, buf)
        cnt[q] = ln[0]
        lists[q, :min(256, ln[0])] = buf[:min(256, ln[0])]
    nb = parity.nb_report(cnt, lists, ref["nb_count"], ref["nb_list"], xp, jm.index, jm.x[sample], h2)
    _say(f"[C3] {prec}: nb={nb}")
    assert nb["ok"], nb
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [0, 3, 7, 12, 16])
def test_config_c3_active_blocks(g6, orc, sess, k):
    """Active blocks of 2^k particles against all 2^20 (the throughput
    sweep), DS, up to 256 sampled i-particles checked."""
    jm = c3_case()
    n = jm.n
    eps2, h2, ti = jm.meta["eps2"], jm.meta["h2"], jm.meta["ti"]
    device_jmem(g6, sess, jm)
    g6.g6mi_set_precision(sess.id, "ds")
    g6.g6mi_set_shape(sess.id, 0, 0)
    g6.g6_set_ti(sess.id, ti)
    slots = workloads.active_set(n, 2 ** k, seed=3)
    _say(f"[C3 k={k}] running")
    dv = device_calc(g6, sess, n, slots, jm.x[slots], jm.v[slots], eps2, h2)
    pick = np.arange(len(slots)) if len(slots) <= 256 else workloads.active_set(len(slots), 256, seed=k)
    xp, vp = orc.predict(ti, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    s = slots[pick]
    ref = orc.force(xp, vp, jm.m, jm.index, jm.x[s], jm.v[s], jm.index[s], eps2, h2, conditioning=True)
    gpu = dict(acc=dv["acc"][pick], jerk=dv["jerk"][pick], pot=dv["pot"][pick])
    rep = parity.force_report(gpu, ref)
    nn = parity.nn_report(dv["nnb"][pick], ref["nn_index"], ref["nn_r2"], xp, jm.index, jm.x[s])
    _say(f"[C3 k={k}] {rep} nn={nn}")
    assert rep["ok"] and nn["ok"]


@pytest.fixture(scope="module")
def c5_case(orc):
    """The config 5 system and the oracle on a sample of it: 1024 binary
    members spread over the binaries' range of semi-major axes and 512
    single stars."""
    jm = workloads.config_c5()
    n = jm.n
    eps2, h2 = jm.meta["eps2"], jm.meta["h2"]
    nb_ = jm.meta["n_binaries"]
    members = np.arange(0, 2 * nb_, max(1, (2 * nb_) // 1024))[:1024]
    singles = workloads.active_set(n - 2 * nb_, 512, 5) + 2 * nb_
    slots = np.unique(np.concatenate([members, singles])).astype(np.int64)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    return jm, slots, ref


def c5_bins(jm, slots):
    """Row groups of the config 5 sample: single stars, and binary members by
    decade of the semi-major axis."""
    nb_ = jm.meta["n_binaries"]
    is_bin = slots < 2 * nb_
    la = np.full(len(slots), np.nan)
    la[is_bin] = np.log10(jm.meta["binary_a"][slots[is_bin] // 2])
    groups = {"single": ~is_bin}
    for lo in (-5, -4):
        groups[f"binary a=1e{lo}..1e{lo + 1}"] = is_bin & (la >= lo) & (la < lo + 1)
    return groups


@pytest.mark.parametrize("prec", ["fp64", "ds", "fp32"])
def test_config_c5_precision_stress(g6, orc, sess, c5_case, prec):
    """Plummer N=2^18 with 5% hard-binary members, translated by 1e4,
    eps = 0, neighbour radius 0.01 (the double-single resolution claim after
    Eq. (3), and the neighbour lists of Sec. 4).  FP64 and DS must meet the
    force tolerances on every single star, and give the oracle's nearest
    neighbours and neighbour lists up to distance ties; FP64 also meets the
    force tolerances on the binary members.  Errors are reported per group:
    single stars and binary members by decade of the semi-major axis (DS
    resolves |x| = 1e4 to about 2^-48 of it, 4e-11, against separations down
    to ~1e-7 at pericentre).  FP32 (ulp 1e-3 at |x| = 1e4) is reported, not
    graded."""
    jm, slots, ref = c5_case
    eps2, h2 = jm.meta["eps2"], jm.meta["h2"]
    sess.load(jm)
    _say(f"[C5] running {prec} on {len(slots)} i-particles")
    gpu = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, prec)
    finite = np.isfinite(gpu["acc"]).all(axis=1) & np.isfinite(gpu["jerk"]).all(axis=1) & np.isfinite(gpu["pot"])
    clean = {k: np.where(np.isfinite(gpu[k]), gpu[k], 0) for k in ("acc", "jerk", "pot")}
    ea, ej, ep = parity.rel_errors(clean, ref)
    xp = ref["_xp"]
    nn = parity.nn_report(gpu["nn_index"], ref["nn_index"], ref["nn_r2"], xp, jm.index, ref["xi"])
    nb = parity.nb_report(gpu["nb_count"], gpu["nb_list"], ref["nb_count"], ref["nb_list"], xp, jm.index,
                          ref["xi"], h2)
    groups = c5_bins(jm, slots)
    for name, g in groups.items():
        if not g.any():
            continue
        _say(f"[C5] {prec} {name} ({int(g.sum())}): nonfinite={int((~finite[g]).sum())} "
             f"acc max={ea[g].max():.2e} median={np.median(ea[g]):.2e}  "
             f"jerk max={ej[g].max():.2e} median={np.median(ej[g]):.2e}  pot max={ep[g].max():.2e}")
    _say(f"[C5] {prec}: nn mismatch={nn['mismatch']} ties={nn['ties']} fail={nn['fail']}; "
         f"neighbour lists fail={nb['fail']} ties={nb['ties']} overflow rows={nb['overflow_rows']}; "
         f"oracle neighbours: {int(ref['nb_count'].sum())} in {int((ref['nb_count'] > 0).sum())} lists")
    if prec == "fp32":
        return
    assert finite.all()
    single = groups["single"]
    keys = ("acc", "jerk", "pot", "acc_abs", "jerk_abs")
    rep_single = parity.force_report({k: clean[k][single] for k in keys[:3]}, {k: ref[k][single] for k in keys})
    assert rep_single["ok"], rep_single
    assert nn["ok"], nn
    assert nb["ok"] and nb["overflow_rows"] == 0, nb
    assert int(ref["nb_count"].sum()) > 0
    if prec == "fp64":
        rep = parity.force_report(clean, ref)
        assert rep["ok"], rep


@pytest.mark.parametrize("prec", ["ds", "fp64"])
@pytest.mark.parametrize("shape", [(0, 0), (64, 3), (512, 2)])
def test_dominant_close_companion(g6, orc, sess, prec, shape):
    """Hard binaries (a = 1e-5 .. 1e-3) inside an untranslated Plummer sphere,
    eps = 0: each member's companion term exceeds the far field by 10^4 -
    10^6.  Float32 partial sums must not swallow the far-field terms that
    follow the companion's (the two-level summation), so DS meets the
    tolerances on binary members and single stars alike."""
    jm = workloads.config_c5(n=2 ** 14, shift=0.0)
    nb = jm.meta["n_binaries"]
    slots = np.concatenate([np.arange(0, 2 * nb, 3), workloads.active_set(jm.n - 2 * nb, 300, 7) + 2 * nb])
    slots = np.unique(slots)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 0.0, 1e-4))
    sess.load(jm)
    gpu = gpu_eval(sess, g6, jm, slots, ref, 0.0, 1e-4, prec, shape)
    rep = assert_parity(gpu, ref, jm, 1e-4, prec, f"binaries shape={shape}")
    if prec == "ds":
        assert rep["acc_max"] < 1e-6, rep


# ------------------------------------------------- spatially ordered DS blocks

SPATIAL_CASES = [(700, 1), (5000, 300), (4097, 4097), (20000, 5000), (65536, 65536)]


@pytest.mark.parametrize("n,ni", SPATIAL_CASES)
def test_spatial_order_parity(g6, orc, sess, n, ni):
    """Double-single with the Morton ordering forced on (far tiles in
    float32 relative to the tile centre): oracle parity of forces, nearest
    neighbours and neighbour lists, including ragged tiles, own-slot tiles
    and blocks smaller than a workgroup; and agreement with the unordered
    kernel to the double-single error level."""
    jm = workloads.random_cluster(n, seed=2000 + n)
    slots = workloads.active_set(n, ni, seed=n)
    eps2, h2 = 1e-4, 0.05
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    try:
        g6.check(sess.id, g6.g6mi_set_spatial(sess.id, 2))
        sp = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds")
        g6.check(sess.id, g6.g6mi_set_spatial(sess.id, 0))
        plain = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds")
    finally:
        g6.g6mi_set_spatial(sess.id, 1)
    assert_parity(sp, ref, jm, h2, "ds", f"spatial N={n} ni={ni}")
    assert_parity(plain, ref, jm, h2, "ds", f"unordered N={n} ni={ni}")
    # the two orders find the same neighbours (up to distance ties)
    xp = ref["_xp"]
    nn = parity.nn_report(sp["nn_index"], plain["nn_index"], parity.r2_to(xp, jm.index, ref["xi"], np.arange(len(slots)),
                                                                           plain["nn_index"]), xp, jm.index, ref["xi"])
    assert nn["ok"], nn


@pytest.mark.parametrize("eps2", [1e-4, 0.0])
def test_spatial_order_without_lists(g6, orc, sess, eps2):
    """The ordered kernel without neighbour lists, where a far tile skips its
    nearest-neighbour work whenever the searches of a wave's particles cannot
    move (no neighbour radius holds it back): oracle parity of forces and
    nearest neighbours, and the same bits as the kernel with lists, whose
    large neighbour radius here keeps most far tiles on the full path (the
    skipped work changes no sum and no search)."""
    jm = workloads.random_cluster(65536, seed=4242)
    slots = workloads.active_set(jm.n, 20000, seed=7)
    h2 = 0.05
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, eps2, h2))
    sess.load(jm)
    try:
        g6.check(sess.id, g6.g6mi_set_spatial(sess.id, 2))
        off = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds", neighbours=False)
        on = gpu_eval(sess, g6, jm, slots, ref, eps2, h2, "ds")
    finally:
        g6.g6mi_set_spatial(sess.id, 1)
    assert_parity(off, ref, jm, h2, "ds", f"spatial without lists eps2={eps2}")
    for k in ("acc", "jerk", "pot", "nn_index", "nn_r2"):
        assert np.array_equal(off[k], on[k]), k


def test_spatial_order_coincident_pairs_at_eps0(g6, orc, sess):
    """Morton ordering forced on, eps = 0, and 40 pairs of particles with the
    same predicted position: each member's nearest neighbour is its partner
    at r^2 = 0.  The kernel starts every particle's nearest-neighbour search
    below an upper bound taken from the record next to its own, and that
    bound must stay above a pair at distance zero.  The other particles keep
    oracle parity of their nearest neighbours (the pairs' forces are not
    finite and are not compared)."""
    rng = np.random.default_rng(88)
    jm = workloads.random_cluster(5000, seed=88)
    a = rng.permutation(jm.n)[:80]
    src, dst = a[:40], a[40:]
    for f in ("x", "v", "a2", "j6", "t"):
        getattr(jm, f)[dst] = getattr(jm, f)[src]
    slots = np.arange(jm.n)
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 0.0, 1e-3))
    sess.load(jm)
    try:
        g6.check(sess.id, g6.g6mi_set_spatial(sess.id, 2))
        gpu = gpu_eval(sess, g6, jm, slots, ref, 0.0, 1e-3, "ds")
    finally:
        g6.g6mi_set_spatial(sess.id, 1)
    assert gpu["nonfinite"]  # the coincident pairs' forces
    for u, w in ((src, dst), (dst, src)):
        assert np.array_equal(gpu["nn_index"][u], jm.index[w])
        # the i-positions are the oracle's predictions, the records the
        # library's: the two can differ in the last bits of float64
        assert np.all(gpu["nn_r2"][a] <= 1e-28)
    # and many pairs meet at exactly zero, the case the search bound must keep
    assert np.sum(gpu["nn_r2"][a] == 0.0) >= 20
    rest = np.setdiff1d(slots, a)
    xp = ref["_xp"]
    nn = parity.nn_report(gpu["nn_index"][rest], ref["nn_index"][rest], ref["nn_r2"][rest], xp, jm.index,
                          ref["xi"][rest])
    assert nn["ok"], nn


def test_spatial_order_neighbour_overflow(g6, orc, sess):
    """Morton ordering forced on with every list overflowing and a shuffled
    index column: partials sit at sorted positions and are mapped back to
    their rows, so the overflow queue must still name rows, and the exact
    pass must keep the 256 smallest indices as the oracle does."""
    rng = np.random.default_rng(62)
    n = 3000
    x = rng.normal(size=(n, 3)) * 0.01
    jm = workloads.make_jmemory(x, rng.normal(size=(n, 3)), np.full(n, 1 / n), meta=dict(ti=0.0),
                                index=rng.permutation(n) * 3 + 7)
    slots = rng.permutation(n)[:900]
    ref = with_xp(orc, jm, oracle_eval(orc, jm, slots, 1e-6, 1.0))
    sess.load(jm)
    try:
        g6.check(sess.id, g6.g6mi_set_spatial(sess.id, 2))
        gpu = gpu_eval(sess, g6, jm, slots, ref, 1e-6, 1.0, "ds")
    finally:
        g6.g6mi_set_spatial(sess.id, 1)
    assert gpu["nb_overflow"]
    assert np.array_equal(gpu["nb_count"], ref["nb_count"])
    assert np.array_equal(gpu["nb_list"], ref["nb_list"])
    forces = {k: v for k, v in gpu.items() if k not in ("nb_count", "nb_list")}
    assert_parity(forces, ref, jm, 1.0, "ds", "spatial overflow")

