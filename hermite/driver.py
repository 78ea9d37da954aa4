"""Block-time-step Hermite integrator (host side).

The scheme is the standard 4th-order predictor-corrector of Makino &
Aarseth (1992), which the paper's library serves (Sec. 2):

* predictor:  every particle is extrapolated by its Taylor series to the
  block time (Eq. (1)-(2)); the j-particles on the GPU, the active
  i-particles here on the host (Sec. 2.1);
* force:      acceleration and jerk of the active block from the backend;
* corrector:  with the new a1, j1 at the end of the step dt,
      a(2) = (-6 (a0 - a1) - dt (4 j0 + 2 j1)) / dt^2
      a(3) = (12 (a0 - a1) + 6 dt (j0 + j1)) / dt^3
      x1 = x_p + a(2) dt^4 / 24 + a(3) dt^5 / 120
      v1 = v_p + a(2) dt^3 / 6  + a(3) dt^4 / 24
* time step:  Aarseth's criterion (cited in Sec. 3.1) with a(2) taken at the
  end of the step, quantised to a power of two that divides the current
  time, growing by at most a factor two per step.

Everything is float64 numpy; the force backend is the only place that
touches the GPU.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _norm(a):
    return np.sqrt(np.sum(a * a, axis=-1))


@dataclass
class HermiteState:
    """Particle state at each particle's own last time t (slot k = particle k)."""

    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    a: np.ndarray = None
    j: np.ndarray = None
    t: np.ndarray = None
    dt: np.ndarray = None
    pot: np.ndarray = None
    index: np.ndarray = None

    def __post_init__(self):
        n = self.m.shape[0]
        self.x = np.array(self.x, dtype=np.float64).reshape(n, 3)
        self.v = np.array(self.v, dtype=np.float64).reshape(n, 3)
        self.m = np.array(self.m, dtype=np.float64)
        for name in ("a", "j"):
            if getattr(self, name) is None:
                setattr(self, name, np.zeros((n, 3)))
        if self.t is None:
            self.t = np.zeros(n)
        if self.dt is None:
            self.dt = np.zeros(n)
        if self.pot is None:
            self.pot = np.zeros(n)
        if self.index is None:
            self.index = np.arange(n, dtype=np.int32)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])

    def predict(self, sel, ti):
        """Taylor extrapolation of the selected particles to time ti."""
        tau = (ti - self.t[sel])[:, None]
        a2 = 0.5 * self.a[sel]
        j6 = self.j[sel] / 6.0
        xp = self.x[sel] + tau * (self.v[sel] + tau * (a2 + tau * j6))
        vp = self.v[sel] + tau * (2.0 * a2 + tau * (3.0 * j6))
        return xp, vp

    def energies(self):
        kin = 0.5 * float(np.sum(self.m * np.sum(self.v * self.v, axis=1)))
        pot = 0.5 * float(np.sum(self.m * self.pot))
        return kin, pot, kin + pot


class G6Backend:
    """Force backend on libg6mi through its GRAPE-6 calls."""

    def __init__(self, n, eps2, h2=0.0, precision="ds", handle=0, neighbour_lists=False):
        import paper_0902_4463_amd as g6
        self.g6 = g6
        self.id = handle
        self.eps2 = float(eps2)
        self.h2 = float(h2)
        self.n = int(n)
        g6.check(handle, g6.g6_open(handle))
        g6.check(handle, g6.g6mi_set_precision(handle, precision))
        g6.check(handle, g6.g6mi_set_neighbour_lists(handle, neighbour_lists))
        self._zero = np.zeros(3)

    def close(self):
        self.g6.g6_close(self.id)

    def set_j(self, st: HermiteState, sel):
        sel = np.asarray(sel)
        self.g6.check(self.id, self.g6.g6mi_set_j_particles(
            self.id, len(sel), sel, st.index[sel], st.t[sel], st.dt[sel], st.m[sel], st.j[sel] / 6.0,
            st.a[sel] / 2.0, st.v[sel], st.x[sel]))

    def force(self, ti, index, xi, vi):
        g6 = self.g6
        ni = len(index)
        h2 = np.full(ni, self.h2)
        g6.g6_set_ti(self.id, ti)
        g6.check(self.id, g6.g6calc_firsthalf(self.id, self.n, ni, index, xi, vi, None, None, None,
                                              self.eps2, h2))
        acc = np.zeros((ni, 3)); jerk = np.zeros((ni, 3)); pot = np.zeros(ni)
        nnb = np.zeros(ni, dtype=np.int32)
        rc = g6.check(self.id, g6.g6calc_lasthalf2(self.id, self.n, ni, index, xi, vi, self.eps2, h2,
                                                   acc, jerk, pot, nnb))
        if rc == g6.WARN:
            raise FloatingPointError("non-finite force from the library")
        return acc, jerk, pot


@dataclass
class StepLog:
    time: float
    n_active: int


class BlockStepIntegrator:
    """Drives a backend with ``set_j(state, sel)`` and
    ``force(ti, index, xi, vi) -> (acc, jerk, pot)``.

    eta: accuracy parameter of the time-step criterion; eta_s: the smaller
    one for the first step (dt = eta_s |a| / |jerk|); dt_max / dt_min bound
    the power-of-two steps.  ``on_step(ti, sel, xi, vi, acc, jerk, pot)`` is
    called after every force evaluation (tests compare with the oracle)."""

    def __init__(self, state: HermiteState, backend, eta=0.01, eta_s=0.01, dt_max=2.0 ** -3,
                 dt_min=2.0 ** -40, on_step=None):
        self.s = state
        self.b = backend
        self.eta = eta
        self.eta_s = eta_s
        self.dt_max = dt_max
        self.dt_min = dt_min
        self.on_step = on_step
        self.time = 0.0
        self.steps = 0
        self.particle_steps = 0
        self.log: list[StepLog] = []
        self._init()

    def _quantise(self, dt):
        """Largest power of two at or below dt (clipped to [dt_min, dt_max]),
        read exactly from the binary exponent: dt = f 2^e with f in [0.5, 1)."""
        dt = np.clip(dt, self.dt_min, self.dt_max)
        _, e = np.frexp(dt)
        return np.ldexp(1.0, e - 1)

    def _init(self):
        s = self.s
        allp = np.arange(s.n)
        s.t[:] = self.time
        s.a[:] = 0.0
        s.j[:] = 0.0
        s.dt[:] = self.dt_max
        self.b.set_j(s, allp)
        acc, jerk, pot = self.b.force(self.time, s.index, s.x, s.v)
        if self.on_step:
            self.on_step(self.time, allp, s.x.copy(), s.v.copy(), acc, jerk, pot)
        s.a[:], s.j[:], s.pot[:] = acc, jerk, pot
        dt = self.eta_s * _norm(acc) / np.maximum(_norm(jerk), 1e-300)
        s.dt[:] = self._quantise(dt)
        self.b.set_j(s, allp)

    def step(self):
        """Advance the block of particles with the earliest t + dt."""
        s = self.s
        tnext = float(np.min(s.t + s.dt))
        sel = np.nonzero(s.t + s.dt == tnext)[0]
        xp, vp = s.predict(sel, tnext)
        acc, jerk, pot = self.b.force(tnext, s.index[sel], xp, vp)
        if self.on_step:
            self.on_step(tnext, sel, xp, vp, acc, jerk, pot)
        dt = (tnext - s.t[sel])[:, None]
        a0, j0 = s.a[sel], s.j[sel]
        a2 = (-6.0 * (a0 - acc) - dt * (4.0 * j0 + 2.0 * jerk)) / dt ** 2
        a3 = (12.0 * (a0 - acc) + 6.0 * dt * (j0 + jerk)) / dt ** 3
        x1 = xp + a2 * dt ** 4 / 24.0 + a3 * dt ** 5 / 120.0
        v1 = vp + a2 * dt ** 3 / 6.0 + a3 * dt ** 4 / 24.0
        # Aarseth criterion with the second derivative at the end of the step
        a2e = a2 + dt * a3
        num = _norm(acc) * _norm(a2e) + _norm(jerk) ** 2
        den = _norm(jerk) * _norm(a3) + _norm(a2e) ** 2
        dt_new = np.sqrt(self.eta * num / np.maximum(den, 1e-300))
        old = s.dt[sel]
        new = old.copy()
        # halve while too long, never below dt_min
        shrink = (dt_new < old) & (old > self.dt_min)
        while np.any(shrink):
            new[shrink] *= 0.5
            shrink = (dt_new < new) & (new > self.dt_min)
        grow = (dt_new >= 2.0 * old) & (np.fmod(tnext, 2.0 * old) == 0.0) & (2.0 * old <= self.dt_max)
        new[grow] = 2.0 * old[grow]
        s.x[sel], s.v[sel], s.a[sel], s.j[sel], s.pot[sel] = x1, v1, acc, jerk, pot
        s.t[sel] = tnext
        s.dt[sel] = new
        self.b.set_j(s, sel)
        self.time = tnext
        self.steps += 1
        self.particle_steps += len(sel)
        self.log.append(StepLog(tnext, len(sel)))
        return tnext, sel

    def run(self, t_end):
        while self.time < t_end:
            self.step()
        return self

    def synchronised(self) -> bool:
        return bool(np.all(self.s.t == self.time))


def kepler_binary(m1=0.5, m2=0.5, a=1.0, e=0.0):
    """Two bodies on a Kepler orbit at pericentre, centre-of-mass frame."""
    mt = m1 + m2
    rp = a * (1.0 - e)
    vp = np.sqrt(mt * (1.0 + e) / rp)
    x = np.array([[-m2 / mt * rp, 0, 0], [m1 / mt * rp, 0, 0]])
    v = np.array([[0, -m2 / mt * vp, 0], [0, m1 / mt * vp, 0]])
    return x, v, np.array([m1, m2])
