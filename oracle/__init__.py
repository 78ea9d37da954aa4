"""CPU float64 oracle for the force evaluation -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the GPU library: the arithmetic lives
in ``g6_oracle.c`` (plain C, built by ``oracle/build.py`` with gcc), and this
module only marshals numpy arrays into it.

Functions (each follows the passage cited in ``g6_oracle.c``):
  predict(...)  -- Sec. 2.2, Eq. (1) and (2): j-particle prediction.
  force(...)    -- acceleration, jerk, potential, nearest neighbour and
                   neighbour list of one block of i-particles (Sec. 2, 2.3,
                   2.5 and 4).
  evaluate(...) -- predict the j-memory, take the active slots' predicted
                   state as the i-block, and run ``force``.
  energies(...) -- kinetic, potential and total energy from a full
                   evaluation (the dE/E diagnostic of Sec. 3.2).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None
NB_CAP_DEFAULT = 256


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_predict.argtypes = [ctypes.c_int64, ctypes.c_double, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_predict.restype = None
        lib.oracle_force.argtypes = [ctypes.c_int64, dp, dp, dp, ip,
                                     ctypes.c_int64, dp, dp, ip, ctypes.c_double, dp,
                                     ctypes.c_int, dp, dp, dp, ip, dp, lp, ip, dp, dp]
        lib.oracle_force.restype = ctypes.c_int64
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _LIB = lib
    return _LIB


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _l(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _vec3(a, n):
    return np.ascontiguousarray(a, dtype=np.float64).reshape(n, 3)


def max_threads() -> int:
    return int(_lib().oracle_max_threads())


def set_threads(n: int) -> None:
    _lib().oracle_set_threads(int(n))


def predict(ti, t, x, v, a2, j6):
    """Predicted positions and velocities of all j-slots at time ti."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    n = t.shape[0]
    x, v, a2, j6 = (_vec3(a, n) for a in (x, v, a2, j6))
    xp = np.empty((n, 3))
    vp = np.empty((n, 3))
    _lib().oracle_predict(n, float(ti), _d(t), _d(x), _d(v), _d(a2), _d(j6), _d(xp), _d(vp))
    return xp, vp


def force(xj, vj, mj, jindex, xi, vi, iindex, eps2, h2=None, nb_cap=NB_CAP_DEFAULT,
          conditioning=False):
    """Force evaluation of i-particles (xi, vi, iindex) by j-particles
    (xj, vj, mj, jindex).  Returns a dict of float64/int arrays; with
    ``conditioning`` also acc_abs / jerk_abs, the sums of the magnitudes of
    the pair terms."""
    mj = np.ascontiguousarray(mj, dtype=np.float64)
    nj = mj.shape[0]
    iindex = np.ascontiguousarray(iindex, dtype=np.int32)
    ni = iindex.shape[0]
    xj, vj = _vec3(xj, nj), _vec3(vj, nj)
    xi, vi = _vec3(xi, ni), _vec3(vi, ni)
    jindex = np.ascontiguousarray(jindex, dtype=np.int32)
    if h2 is None:
        h2 = np.zeros(ni)
    h2 = np.ascontiguousarray(np.broadcast_to(np.asarray(h2, dtype=np.float64), (ni,)))
    out = dict(
        acc=np.empty((ni, 3)), jerk=np.empty((ni, 3)), pot=np.empty(ni),
        nn_index=np.empty(ni, dtype=np.int32), nn_r2=np.empty(ni),
        nb_count=np.empty(ni, dtype=np.int64),
        nb_list=np.empty((ni, max(nb_cap, 0)), dtype=np.int32),
    )
    if conditioning:
        out["acc_abs"], out["jerk_abs"] = np.empty(ni), np.empty(ni)
    ndeg = _lib().oracle_force(
        nj, _d(xj), _d(vj), _d(mj), _i(jindex), ni, _d(xi), _d(vi), _i(iindex),
        float(eps2), _d(h2), int(nb_cap), _d(out["acc"]), _d(out["jerk"]), _d(out["pot"]),
        _i(out["nn_index"]), _d(out["nn_r2"]), _l(out["nb_count"]), _i(out["nb_list"]),
        _d(out["acc_abs"]) if conditioning else None, _d(out["jerk_abs"]) if conditioning else None)
    out["n_degenerate"] = int(ndeg)
    return out


def evaluate(jm, ti, slots, eps2, h2=None, nb_cap=NB_CAP_DEFAULT, conditioning=False):
    """One block step's force evaluation on a j-memory (``workloads.JMemory``):
    every j-slot is predicted to ti, the active ``slots`` take their predicted
    state as i-particles, and their forces are summed over all other slots."""
    xp, vp = predict(ti, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    slots = np.asarray(slots, dtype=np.int64)
    res = force(xp, vp, jm.m, jm.index, xp[slots], vp[slots], jm.index[slots],
                eps2, h2, nb_cap, conditioning)
    res["xi"], res["vi"] = xp[slots], vp[slots]
    return res


def energies(m, v, pot):
    """Kinetic, potential and total energy: K = 1/2 sum m v^2 and
    W = 1/2 sum m phi (each pair counted once)."""
    m = np.asarray(m, dtype=np.float64)
    kin = 0.5 * float(np.sum(m * np.sum(np.asarray(v) ** 2, axis=1)))
    wpot = 0.5 * float(np.sum(m * np.asarray(pot)))
    return kin, wpot, kin + wpot
