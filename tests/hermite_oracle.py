"""Force backend for the Hermite driver that uses the float64 CPU oracle
(test infrastructure: it keeps its own copy of the j-memory, predicts it with
the oracle's predictor and sums with the oracle's force routine)."""

import numpy as np

import oracle
from tests import parity


class OracleBackend:
    def __init__(self, n, eps2, h2=0.0):
        self.eps2 = float(eps2)
        self.h2 = float(h2)
        self.x = np.zeros((n, 3)); self.v = np.zeros((n, 3))
        self.a2 = np.zeros((n, 3)); self.j6 = np.zeros((n, 3))
        self.t = np.zeros(n); self.m = np.zeros(n)
        self.index = np.arange(n, dtype=np.int32)

    def set_j(self, st, sel):
        sel = np.asarray(sel)
        self.x[sel] = st.x[sel]; self.v[sel] = st.v[sel]
        self.a2[sel] = st.a[sel] / 2.0; self.j6[sel] = st.j[sel] / 6.0
        self.t[sel] = st.t[sel]; self.m[sel] = st.m[sel]; self.index[sel] = st.index[sel]

    def jmemory(self, ti):
        return oracle.predict(ti, self.t, self.x, self.v, self.a2, self.j6)

    def force(self, ti, index, xi, vi, conditioning=False):
        xp, vp = self.jmemory(ti)
        r = oracle.force(xp, vp, self.m, self.index, xi, vi, index, self.eps2, self.h2,
                         conditioning=conditioning)
        if conditioning:
            return r
        return r["acc"], r["jerk"], r["pot"]

    def close(self):
        pass


class Shadowed:
    """GPU backend plus an oracle copy of the same j-memory; each force call
    is compared with the oracle (all i, or a seeded sample of ``cap``)."""

    def __init__(self, n, eps2, precision, cap=None, handle=2):
        from hermite import G6Backend
        self.gpu = G6Backend(n, eps2, precision=precision, handle=handle)
        self.ref = OracleBackend(n, eps2)
        self.cap = cap
        self.worst = dict(acc=0.0, jerk=0.0, pot=0.0)
        self.fails = []
        self.checked = 0
        self.rng = np.random.default_rng(0)
        self.record = []  # per force call: (ti, ni, checked, acc_max, jerk_max, pot_max, conditioned)
        self.keep_fail_inputs = False  # keep the inputs and results of the first failing calls
        self.fail_inputs = []

    def set_j(self, st, sel):
        self.gpu.set_j(st, sel)
        self.ref.set_j(st, sel)

    def force(self, ti, index, xi, vi):
        acc, jerk, pot = self.gpu.force(ti, index, xi, vi)
        pick = np.arange(len(index))
        if self.cap is not None and len(index) > self.cap:
            pick = np.sort(self.rng.choice(len(index), self.cap, replace=False))
        r = self.ref.force(ti, index[pick], xi[pick], vi[pick], conditioning=True)
        rep = parity.force_report(dict(acc=acc[pick], jerk=jerk[pick], pot=pot[pick]), r)
        self.checked += len(pick)
        for k, key in (("acc", "acc_max"), ("jerk", "jerk_max"), ("pot", "pot_max")):
            self.worst[k] = max(self.worst[k], rep[key])
        if not rep["ok"]:
            self.fails.append((ti, len(index), rep))
            if self.keep_fail_inputs and len(self.fail_inputs) < 4:
                xp, vp = self.ref.jmemory(ti)
                self.fail_inputs.append(dict(ti=ti, index=np.asarray(index)[pick], xi=xi[pick], vi=vi[pick],
                                             acc=acc[pick], jerk=jerk[pick], pot=pot[pick], ref_acc=r["acc"],
                                             ref_jerk=r["jerk"], ref_pot=r["pot"], xj=xp, vj=vp, mj=self.ref.m.copy(),
                                             jindex=self.ref.index.copy()))
        self.record.append((float(ti), len(index), len(pick), rep["acc_max"], rep["jerk_max"], rep["pot_max"],
                            rep["acc_conditioned"] + rep["jerk_conditioned"]))
        return acc, jerk, pot

    def close(self):
        self.gpu.close()
