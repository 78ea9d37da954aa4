"""Hermite block-step integrations driven by libg6mi (GPU), with every force
evaluation checked against the float64 oracle on the same predicted state."""

import collections
import sys

import numpy as np
import pytest

import workloads
from hermite import BlockStepIntegrator, HermiteState
from tests.hermite_oracle import OracleBackend, Shadowed

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def energy_drift(st, it, t_end):
    e0 = st.energies()[2]
    it.run(t_end)
    assert it.synchronised()
    return (st.energies()[2] - e0) / e0


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_config_c1_hermite_run(prec):
    """Equal-mass Plummer N=1024, eps = 1/64, eta = 0.01, to t = 1/8 with
    individual block steps; every step checked in full."""
    jm = workloads.config_c1()
    eps2 = jm.meta["eps2"]
    st = HermiteState(jm.x, jm.v, jm.m)
    b = Shadowed(jm.n, eps2, prec)
    try:
        it = BlockStepIntegrator(st, b, eta=0.01, dt_max=0.125)
        de = energy_drift(st, it, 0.125)
    finally:
        b.close()
    # the same run on the oracle alone
    st2 = HermiteState(jm.x, jm.v, jm.m)
    it2 = BlockStepIntegrator(st2, OracleBackend(jm.n, eps2), eta=0.01, dt_max=0.125)
    de2 = energy_drift(st2, it2, 0.125)
    hist = collections.Counter(int(np.log2(s.n_active)) for s in it.log)
    _say(f"[C1 hermite {prec}] dE/E={de:.3e} (oracle run {de2:.3e}) block steps={it.steps} "
         f"particle steps={it.particle_steps} checked={b.checked} worst={b.worst} "
         f"log2(block) histogram={sorted(hist.items())}")
    assert not b.fails, b.fails[:3]
    assert abs(de) < 1e-6 and abs(de) < 10 * abs(de2) + 1e-8
    if prec == "fp64":
        assert abs(de - de2) < 1e-10


@pytest.mark.parametrize("prec", ["ds", "fp64"])
def test_config_c2_hermite_segment(prec):
    """Equal-mass Plummer N=32768, eps = 1e-4, eta = 0.01: the first 2^-7
    time units, block steps checked on up to 256 sampled i-particles."""
    jm = workloads.config_c2()
    eps2 = jm.meta["eps2"]
    st = HermiteState(jm.x, jm.v, jm.m)
    b = Shadowed(jm.n, eps2, prec, cap=256)
    try:
        it = BlockStepIntegrator(st, b, eta=0.01, dt_max=2.0 ** -4)
        it.run(2.0 ** -7)
    finally:
        b.close()
    _say(f"[C2 hermite {prec}] t={it.time} block steps={it.steps} particle steps={it.particle_steps} "
         f"checked={b.checked} worst={b.worst} mean block={it.particle_steps / it.steps:.1f}")
    assert not b.fails, b.fails[:3]
