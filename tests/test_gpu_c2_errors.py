"""Config 2: equal-mass Plummer N = 32768, eps = 1e-4, eta = 0.01, Hermite
block steps driven by libg6mi, every force call compared with the float64
oracle on the same predicted state (Sec. 3.2 runs N = 32k Plummer models
through the library with individual block time steps).

Each call's i-particles are checked in full up to 1024, else on a seeded
sample of 1024.  The double-single run goes to t = 1 in eight tests of 1/8
each on one integrator (a module fixture carries it from test to test); the
float64 run goes to t = 1/8."""

import sys
import time

import numpy as np
import pytest

import workloads
from hermite import BlockStepIntegrator, HermiteState
from tests.hermite_oracle import Shadowed

pytestmark = pytest.mark.gpu

CAP = 1024


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class C2Run:
    def __init__(self, prec, handle):
        self.prec = prec
        jm = workloads.config_c2()
        self.st = HermiteState(jm.x, jm.v, jm.m)
        self.b = Shadowed(jm.n, jm.meta["eps2"], prec, cap=CAP, handle=handle)
        self.it = BlockStepIntegrator(self.st, self.b, eta=0.01, dt_max=2.0 ** -4)
        self.e0 = self.st.energies()[2]
        self.marks = []
        self.w0 = time.perf_counter()

    def advance(self, t):
        self.it.run(t)
        de = (self.st.energies()[2] - self.e0) / self.e0
        self.marks.append((t, de))
        _say(f"[C2 {self.prec}] t={self.it.time:.4f} dE/E={de:.3e} block steps={self.it.steps} "
             f"calls={len(self.b.record)} worst={self.b.worst} fails={len(self.b.fails)} "
             f"{time.perf_counter() - self.w0:.0f} s")
        return de

    def summary(self):
        rec = np.array([r[1:] for r in self.b.record], dtype=float)
        ni, checked, acc, jerk, pot, cond = rec.T
        _say(f"[C2 {self.prec}] to t={self.it.time}: block steps={self.it.steps} "
             f"particle steps={self.it.particle_steps} force calls={len(self.b.record)} "
             f"particles checked={int(checked.sum())} failing calls={len(self.b.fails)} "
             f"worst acc={acc.max():.2e} jerk={jerk.max():.2e} pot={pot.max():.2e} "
             f"p99 of per-call worst acc={np.percentile(acc, 99):.2e} conditioned results={int(cond.sum())} "
             f"{time.perf_counter() - self.w0:.0f} s")
        _say(f"[C2 {self.prec}] dE/E at t=k/8: " + ", ".join(f"{t:.3f}: {de:.3e}" for t, de in self.marks))


@pytest.fixture(scope="module")
def c2_ds():
    r = C2Run("ds", handle=5)
    yield r
    r.b.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", range(1, 9))
def test_config_c2_ds_every_call_against_oracle(c2_ds, k):
    """Double-single forces of every block step from t = (k-1)/8 to k/8."""
    if c2_ds.b.fails or (k > 1 and not c2_ds.marks):
        pytest.fail("an earlier segment of the run failed")
    de = c2_ds.advance(k / 8)
    assert not c2_ds.b.fails, c2_ds.b.fails[:3]
    assert abs(de) < 1e-4
    if k == 8:
        c2_ds.summary()
        assert c2_ds.it.synchronised() and c2_ds.it.time == 1.0
        assert len(c2_ds.marks) == 8


@pytest.mark.timeout(600)
def test_config_c2_fp64_to_t_eighth_every_call_against_oracle():
    r = C2Run("fp64", handle=6)
    try:
        r.advance(0.125)
        r.summary()
    finally:
        r.b.close()
    assert not r.b.fails, r.b.fails[:3]
    # float64 forces: every checked particle far inside the tolerances
    assert r.b.worst["acc"] < 1e-10 and r.b.worst["jerk"] < 1e-9 and r.b.worst["pot"] < 1e-11, r.b.worst
