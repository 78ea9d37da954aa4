"""Device-resident block steps (g6mi_hermite_*) against the host-side
integrator.

The integrator inside the library follows the host driver
(hermite/driver.py) formula by formula; with the same force kernel
precision both take the same block sequence, and their states agree up to
the rounding of the force sums.  The host driver on the float64 oracle
(tests/hermite_oracle.py) pins the first steps to the oracle's forces, and a
Kepler orbit pins the scheme to a closed form.
"""

import sys

import numpy as np
import pytest

import workloads
from hermite.driver import BlockStepIntegrator, G6Backend, HermiteState, kepler_binary
from tests.hermite_oracle import OracleBackend

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


def device_run(g6, hid, x, v, m, eps2, eta, dt_max, t_end=None, max_steps=1 << 40, prec="ds", index=None):
    n = len(m)
    index = np.arange(n) if index is None else index
    g6.check(hid, g6.g6_open(hid))
    try:
        g6.check(hid, g6.g6mi_set_precision(hid, prec))
        g6.check(hid, g6.g6mi_set_neighbour_lists(hid, False))
        g6.check(hid, g6.g6mi_set_j_particles(hid, n, np.arange(n), index, np.zeros(n), None, m, np.zeros((n, 3)),
                                              np.zeros((n, 3)), v, x))
        g6.check(hid, g6.g6mi_hermite_init(hid, n, eps2, 0.0, eta, 0.01, dt_max, 2.0 ** -40), allow_warn=False)
        res = dict(init=g6.g6mi_hermite_state(hid, n))
        rc, t, bsteps, psteps = g6.g6mi_hermite_advance(hid, t_end if t_end is not None else 1e30, max_steps)
        g6.check(hid, rc, allow_warn=False)
        res.update(t=t, block_steps=bsteps, particle_steps=psteps, state=g6.g6mi_hermite_state(hid, n))
        return res
    finally:
        g6.g6_close(hid)


def host_run(backend, x, v, m, eta, dt_max, t_end=None, steps=None):
    st = HermiteState(x, v, m)
    it = BlockStepIntegrator(st, backend, eta=eta, dt_max=dt_max)
    if steps is not None:
        for _ in range(steps):
            it.step()
    else:
        it.run(t_end)
    return it, st


def energy(m, v, pot):
    return 0.5 * float(np.sum(m * np.sum(v * v, axis=1))) + 0.5 * float(np.sum(m * pot))


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_device_steps_match_host_driver(g6, prec):
    """Config 1 (N=1024, eps=1/64, eta=0.01) to t=1/8: the same block
    sequence as the host driver on the library's host path, the same final
    state up to force-sum rounding, the same energy error."""
    jm = workloads.config_c1()
    eps2 = jm.meta["eps2"]
    dev = device_run(g6, 5, jm.x, jm.v, jm.m, eps2, 0.01, 0.125, t_end=0.125, prec=prec)
    back = G6Backend(jm.n, eps2, precision=prec, handle=6)
    try:
        it, st = host_run(back, jm.x, jm.v, jm.m, 0.01, 0.125, t_end=0.125)
    finally:
        back.close()
    s = dev["state"]
    _say(f"[device hermite {prec}] blocks device={dev['block_steps']} host={it.steps} "
         f"particle steps device={dev['particle_steps']} host={it.particle_steps}")
    assert dev["t"] == 0.125 and np.all(s["t"] == 0.125)
    dx = np.abs(s["x"] - st.x).max()
    dv = np.abs(s["v"] - st.v).max()
    e0 = energy(jm.m, dev["init"]["v"], dev["init"]["pot"])
    de_dev = (energy(jm.m, s["v"], s["pot"]) - e0) / e0
    de_host = (st.energies()[2] - e0) / e0
    _say(f"[device hermite {prec}] max|dx|={dx:.2e} max|dv|={dv:.2e} dE/E device={de_dev:.3e} host={de_host:.3e}")
    assert abs(de_dev) < 1e-6
    if prec == "fp64":
        # forces equal to float64 rounding: the same decisions, the same state
        assert dev["block_steps"] == it.steps and dev["particle_steps"] == it.particle_steps
        assert dx < 1e-9 and dv < 1e-8 and abs(de_dev - de_host) < 1e-9
    else:
        # the batched and single-system kernels round the float64 split sums
        # in different orders; over 300 block steps a time-step decision at a
        # power-of-two boundary may go the other way for a few particles
        assert dev["block_steps"] == pytest.approx(it.steps, rel=0.01)
        assert dev["particle_steps"] == pytest.approx(it.particle_steps, rel=1e-3)
        assert dx < 1e-6 and abs(de_dev - de_host) < 1e-8


def test_device_first_steps_against_oracle(g6):
    """Twenty block steps of config 1 inside the library (float64 variant)
    against the host driver on the float64 CPU oracle: the same blocks and
    states within the float64 rounding of the force sums."""
    jm = workloads.config_c1()
    eps2 = jm.meta["eps2"]
    dev = device_run(g6, 5, jm.x, jm.v, jm.m, eps2, 0.01, 0.125, max_steps=20, prec="fp64")
    it, st = host_run(OracleBackend(jm.n, eps2), jm.x, jm.v, jm.m, 0.01, 0.125, steps=20)
    s = dev["state"]
    assert dev["block_steps"] == 20 == it.steps
    assert dev["particle_steps"] == it.particle_steps
    assert np.array_equal(s["t"], st.t) and np.array_equal(s["dt"], st.dt)
    for name, a, b, tol in (("x", s["x"], st.x, 1e-12), ("v", s["v"], st.v, 1e-11), ("acc", s["acc"], st.a, 1e-10),
                            ("jerk", s["jerk"], st.j, 1e-9)):
        err = np.abs(a - b).max() / np.abs(b).max()
        _say(f"[device vs oracle] {name}: {err:.2e}")
        assert err < tol, name


def test_device_kepler_orbit(g6):
    """A circular binary over one period returns to its start; halving eta^2
    (dt / 2) shrinks the miss by about 2^4 (4th order)."""
    x, v, m = kepler_binary(e=0.0)
    period = 2 * np.pi
    misses = []
    for eta in (4e-4, 1e-4):
        # integrate to the time grid point nearest one period, then compare
        # with the closed-form position there
        dev = device_run(g6, 5, x, v, m, 0.0, eta, 2.0 ** -5, t_end=period, prec="fp64")
        t = dev["t"]
        ang = t  # angular velocity 1 for a = 1, M = 1
        want = np.array([[-0.5 * np.cos(ang), -0.5 * np.sin(ang), 0], [0.5 * np.cos(ang), 0.5 * np.sin(ang), 0]])
        misses.append(np.abs(dev["state"]["x"] - want).max())
        _say(f"[kepler] eta={eta} t={t:.6f} steps={dev['block_steps']} miss={misses[-1]:.3e}")
    assert misses[0] < 1e-6
    assert misses[0] / misses[1] > 8.0


def test_device_calls_check_state_and_arguments(g6):
    jm = workloads.random_cluster(100, seed=3)
    hid = 5
    g6.check(hid, g6.g6_open(hid))
    try:
        assert g6.g6mi_hermite_advance(hid, 1.0, 10)[0] == g6.ESTATE
        n = jm.n
        # unequal times are refused
        g6.check(hid, g6.g6mi_set_j_particles(hid, n, np.arange(n), jm.index, jm.t, None, jm.m, jm.j6, jm.a2, jm.v,
                                              jm.x))
        assert g6.g6mi_hermite_init(hid, n, 1e-4, 0.0, 0.01, 0.01, 0.125, 2.0 ** -40) == g6.EINVAL
        g6.check(hid, g6.g6mi_set_j_particles(hid, n, np.arange(n), jm.index, np.zeros(n), None, jm.m, jm.j6, jm.a2,
                                              jm.v, jm.x))
        assert g6.g6mi_hermite_init(hid, n + 1, 1e-4, 0.0, 0.01, 0.01, 0.125, 2.0 ** -40) == g6.EINVAL
        assert g6.g6mi_hermite_init(hid, n, 1e-4, 0.0, -1.0, 0.01, 0.125, 2.0 ** -40) == g6.EINVAL
        # dt_max = 2^-6: every particle ends exactly at t = 2^-6
        g6.check(hid, g6.g6mi_hermite_init(hid, n, 1e-4, 0.0, 0.01, 0.01, 2.0 ** -6, 2.0 ** -40))
        rc, t, b, p = g6.g6mi_hermite_advance(hid, 1.0, 0)
        assert rc == g6.OK and t == 0.0 and b == 0 and p == 0
        rc, t, b, p = g6.g6mi_hermite_advance(hid, 2.0 ** -6, 1 << 30)
        assert rc == g6.OK and t == 2.0 ** -6 and b > 0 and p >= n
        st = g6.g6mi_hermite_state(hid, n)
        assert np.all(st["t"] == 2.0 ** -6)
        # the j-memory now holds the integrated state: a host-path force
        # call sees the new positions
        acc = np.zeros((n, 3)); jerk = np.zeros((n, 3)); pot = np.zeros(n)
        g6.g6_set_ti(hid, 2.0 ** -6)
        g6.check(hid, g6.g6calc_firsthalf(hid, n, n, jm.index, st["x"], st["v"], None, None, None, 1e-4, None))
        g6.check(hid, g6.g6calc_lasthalf(hid, n, n, jm.index, st["x"], st["v"], 1e-4, None, acc, jerk, pot))
        assert np.abs(acc - st["acc"]).max() <= 1e-5 * np.abs(st["acc"]).max()
    finally:
        g6.g6_close(hid)
