"""The host-side Hermite block-step driver, run on the CPU oracle backend."""

import numpy as np
import pytest

import workloads
from hermite import BlockStepIntegrator, HermiteState, kepler_binary
from tests.hermite_oracle import OracleBackend


def run_kepler(eta, e, t_end):
    x, v, m = kepler_binary(0.5, 0.5, 1.0, e)
    st = HermiteState(x, v, m)
    b = OracleBackend(2, 0.0)
    it = BlockStepIntegrator(st, b, eta=eta, eta_s=eta / 4, dt_max=2.0 ** -3)
    e0 = None
    it.run(0.0)
    kin0 = 0.5 * np.sum(m * np.sum(v * v, axis=1))
    pot0 = -m[0] * m[1] / np.linalg.norm(x[0] - x[1])
    e0 = kin0 + pot0
    it.run(t_end)
    xs, vs = st.x, st.v
    kin = 0.5 * np.sum(m * np.sum(vs * vs, axis=1))
    pot = -m[0] * m[1] / np.linalg.norm(xs[0] - xs[1])
    return abs((kin + pot - e0) / e0), it


@pytest.mark.parametrize("e", [0.0, 0.5])
def test_kepler_energy_error_is_fourth_order(e):
    """Hermite is a 4th-order scheme: over a fixed time the energy error
    falls at least as (number of steps)^-4 (the circular orbit does better)."""
    t_end = 4.0
    (e1, it1), (e2, it2) = (run_kepler(eta, e, t_end) for eta in (0.02, 0.005))
    order = np.log(e1 / e2) / np.log(it2.steps / it1.steps)
    assert order > 3.6, (e1, e2, it1.steps, it2.steps, order)
    assert e2 < 1e-6


def test_kepler_orbit_returns():
    """A circular orbit (period 2 pi for a = 1, M = 1) comes back to its
    start after one period, to the integration accuracy."""
    x, v, m = kepler_binary(0.5, 0.5, 1.0, 0.0)
    st = HermiteState(x, v, m)
    it = BlockStepIntegrator(st, OracleBackend(2, 0.0), eta=0.002, eta_s=0.0005, dt_max=2.0 ** -6)
    period = 2 * np.pi
    while it.time + st.dt[0] <= period:
        it.step()
    # advance the last fraction with the Taylor predictor of the state
    xp, _ = st.predict(np.arange(2), period)
    assert np.allclose(xp, x, atol=1e-6)


def test_block_steps_are_powers_of_two_and_commensurate():
    jm = workloads.random_cluster(64, seed=3, mass_kind="equal")
    st = HermiteState(jm.x, jm.v, jm.m)
    it = BlockStepIntegrator(st, OracleBackend(64, 1e-4), eta=0.02, dt_max=2.0 ** -4)
    for _ in range(60):
        t, sel = it.step()
        dts = st.dt
        assert np.all(np.log2(dts) == np.round(np.log2(dts)))
        assert np.all(np.fmod(st.t, st.dt) == 0.0)
        assert np.all(st.t[sel] == t)
    assert len(set(n.n_active for n in it.log)) > 1  # genuinely individual blocks


def test_small_plummer_conserves_energy_and_momentum():
    jm = workloads.random_cluster(128, seed=5, mass_kind="equal")
    eps2 = 2.0 ** -12
    st = HermiteState(jm.x, jm.v, jm.m)
    b = OracleBackend(128, eps2)
    it = BlockStepIntegrator(st, b, eta=0.01, dt_max=2.0 ** -4)
    e0 = st.energies()[2]
    p0 = (st.m[:, None] * st.v).sum(axis=0)
    it.run(2.0 ** -4)
    assert it.synchronised()
    # potentials of the final synchronised block are all at time t
    e1 = st.energies()[2]
    assert abs((e1 - e0) / e0) < 1e-6
    # individual steps break exact momentum conservation only at the integration-error level
    assert np.allclose((st.m[:, None] * st.v).sum(axis=0), p0, atol=1e-8)


class ConstantForce:
    """Backend returning the same acceleration and jerk (|jerk| = 10^6 |a|)
    at every call.  The corrector's derivatives are then a2 = -6 j / dt and
    a3 = 12 j / dt^2, and the Aarseth step comes out near
    sqrt(eta dt^2 / 48), far below dt_min once dt is there."""

    def __init__(self, n):
        self.n = n

    def set_j(self, st, sel):
        pass

    def force(self, ti, index, xi, vi):
        k = len(index)
        return np.ones((k, 3)), np.full((k, 3), 1e6), -np.ones(k)


def test_step_never_drops_below_dt_min():
    """A particle at dt_min whose Aarseth step is shorter still stays at
    dt_min: the step is halved only while it is above dt_min."""
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    st = HermiteState(x, np.zeros((2, 3)), np.ones(2))
    dt_min = 2.0 ** -20
    # first step eta_s |a| / |jerk| = 1e-4, quantised to 2^-14
    it = BlockStepIntegrator(st, ConstantForce(2), eta=0.01, eta_s=100.0, dt_max=2.0 ** -3, dt_min=dt_min)
    assert np.all(st.dt == 2.0 ** -14)
    times = [it.time]
    for _ in range(12):
        it.step()
        times.append(it.time)
        assert np.all(st.dt >= dt_min), st.dt
    assert np.all(st.dt == dt_min)
    assert np.all(np.diff(times)[-5:] == dt_min)
