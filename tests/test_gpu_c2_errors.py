"""Config 2: equal-mass Plummer N = 32768, eps = 1e-4, eta = 0.01, Hermite
block steps driven by libg6mi, every force call compared with the float64
oracle on the same predicted state (Sec. 3.2 runs N = 32k Plummer models
through the library with individual block time steps).

Each call's i-particles are checked in full up to 1024, else on a seeded
sample of 1024.  The double-single run goes to t = 1, the float64 run to
t = 1/8.  Progress goes to stdout as the run advances (it takes minutes)."""

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


def run_c2(prec, t_end):
    jm = workloads.config_c2()
    eps2 = jm.meta["eps2"]
    st = HermiteState(jm.x, jm.v, jm.m)
    b = Shadowed(jm.n, eps2, prec, cap=CAP)
    w0 = time.perf_counter()
    marks = []
    try:
        it = BlockStepIntegrator(st, b, eta=0.01, dt_max=2.0 ** -4)
        e0 = st.energies()[2]
        k = 1
        while k / 64 <= t_end + 1e-12:
            it.run(k / 64)
            if k % 8 == 0:
                de = (st.energies()[2] - e0) / e0
                marks.append((k / 64, de))
                _say(f"[C2 {prec}] t={it.time:.4f} dE/E={de:.3e} block steps={it.steps} calls={len(b.record)} "
                     f"worst={b.worst} fails={len(b.fails)} {time.perf_counter() - w0:.0f} s")
            k += 1
    finally:
        b.close()
    rec = np.array([r[1:] for r in b.record], dtype=float)
    ni, checked, acc, jerk, pot, cond = rec.T
    _say(f"[C2 {prec}] to t={t_end}: block steps={it.steps} particle steps={it.particle_steps} "
         f"force calls={len(b.record)} particles checked={int(checked.sum())} failing calls={len(b.fails)} "
         f"worst acc={acc.max():.2e} jerk={jerk.max():.2e} pot={pot.max():.2e} "
         f"p99 of per-call worst acc={np.percentile(acc, 99):.2e} conditioned results={int(cond.sum())} "
         f"{time.perf_counter() - w0:.0f} s")
    _say(f"[C2 {prec}] dE/E at t=k/8: " + ", ".join(f"{t:.3f}: {de:.3e}" for t, de in marks))
    return it, b, marks


@pytest.mark.timeout(900)
def test_config_c2_ds_to_t1_every_call_against_oracle():
    it, b, marks = run_c2("ds", 1.0)
    assert it.synchronised() and it.time == 1.0
    assert not b.fails, b.fails[:3]
    assert len(marks) == 8 and all(abs(de) < 1e-4 for _, de in marks)


@pytest.mark.timeout(600)
def test_config_c2_fp64_to_t_eighth_every_call_against_oracle():
    it, b, marks = run_c2("fp64", 0.125)
    assert not b.fails, b.fails[:3]
    # float64 forces: every checked particle far inside the tolerances
    assert b.worst["acc"] < 1e-10 and b.worst["jerk"] < 1e-9 and b.worst["pot"] < 1e-11, b.worst
    assert len(marks) == 1
