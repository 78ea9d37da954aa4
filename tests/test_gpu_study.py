"""The accuracy study (energy error against the step parameter eta and the
mean block size, Sec. 3.2 and 3.1) as its script runs it, with the block
steps inside the library, against the host-side Hermite driver on the
float64 oracle: config 1 (equal-mass Plummer N = 1024, eps = 1/64) to
t = 1/8 at two values of eta."""

import sys

import numpy as np
import pytest

import workloads
from hermite import BlockStepIntegrator, HermiteState
from hermite import study
from tests.hermite_oracle import OracleBackend

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host_oracle_run(jm, eta, t_end, dt_max):
    eps2 = jm.meta["eps2"]
    st = HermiteState(jm.x, jm.v, jm.m)
    it = BlockStepIntegrator(st, OracleBackend(jm.n, eps2), eta=eta, eta_s=min(eta, 0.01), dt_max=dt_max)
    e0 = st.energies()[2]
    it.run(t_end)
    assert it.synchronised()
    return (st.energies()[2] - e0) / e0, it.steps, it.particle_steps


@pytest.mark.parametrize("eta", [0.01, 0.003])
def test_study_config_c1_against_host_driver_on_oracle(eta):
    import paper_0902_4463_amd as g6
    jm = workloads.config_c1()
    t_end = dt_max = 0.125
    de_ref, steps_ref, psteps_ref = host_oracle_run(jm, eta, t_end, dt_max)
    mean_ref = psteps_ref / steps_ref
    rows = {}
    for prec in ("fp64", "ds"):
        r = study.run_one(g6, 3, jm, eta, prec, t_end, dt_max, 400000)
        rows[prec] = r
        _say(f"[study C1 eta={eta}] {prec}: dE/E={r['energy'][-1]['dE_over_E']:.6e} block steps={r['block_steps']} "
             f"mean block={r['mean_block']:.2f}  host driver on the oracle: dE/E={de_ref:.6e} "
             f"block steps={steps_ref} mean block={mean_ref:.2f}")
        assert not r["capped"] and r["t_reached"] == t_end
        assert [m["t"] for m in r["energy"]] == [0.125]
    fp, ds = rows["fp64"], rows["ds"]
    # float64 forces inside the library: the energy error of the host run
    assert abs(fp["energy"][-1]["dE_over_E"] - de_ref) < 1e-9
    assert abs(fp["mean_block"] - mean_ref) <= 0.01 * mean_ref
    # double-single: float32 pair terms add an energy error of the order of
    # the paper's floor for its double-single library (about 1e-9, Sec. 3.2)
    assert abs(ds["energy"][-1]["dE_over_E"] - de_ref) < 1e-8
    assert abs(ds["mean_block"] - mean_ref) <= 0.05 * mean_ref
    assert np.isfinite(ds["energy"][-1]["dE_over_E"])
