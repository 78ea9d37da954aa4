"""Force backend for the Hermite driver that uses the float64 CPU oracle
(test infrastructure: it keeps its own copy of the j-memory, predicts it with
the oracle's predictor and sums with the oracle's force routine)."""

import numpy as np

import oracle


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
