"""Python binding of libg6mi, the gfx950 direct-summation force library.

This module only marshals arguments: every step of a force calculation
(j-prediction, pair interaction, reduction, neighbour selection) runs in the
HIP kernels of ``libg6mi.so``.  The functions keep the names of the C ABI in
``include/g6mi.h``.  Host arrays are numpy float64 / int32 arrays; device
buffers (for the ``g6mi_*_device`` calls) are torch tensors on the GPU or raw
integer addresses, and streams are ``torch.cuda.Stream`` objects or raw
``hipStream_t`` handles.  PyTorch is used only for device memory and streams.

The library is loaded on the first call; a missing or stale ``libg6mi.so``
raises ``ImportError`` there: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB as LIB_PATH

_lib = None

# constants mirrored from include/g6mi.h
NB_MAX = 256
NPIPES_DEFAULT = 256
NI_MAX = 1 << 24
NJ_MAX = 1 << 26
MAX_HANDLES = 1024
PREC_FP32, PREC_DS, PREC_FP64 = 0, 1, 2
PRECISIONS = {"fp32": PREC_FP32, "ds": PREC_DS, "fp64": PREC_FP64}
OK, WARN, EINVAL, ESTATE, EDEVICE, ENOMEM = 0, 1, -1, -2, -3, -4
FLAG_NONFINITE, FLAG_NB_OVERFLOW, FLAG_BAD_CLUSTER = 1, 2, 4

# struct g6mi_cluster (32 bytes, no padding)
CLUSTER_DTYPE = np.dtype([("joff", "<i4"), ("nj", "<i4"), ("ioff", "<i4"), ("ni", "<i4"),
                          ("ti", "<f8"), ("eps2", "<f8")])
assert CLUSTER_DTYPE.itemsize == 32


class BatchTuning(ctypes.Structure):
    """struct g6mi_batch_tuning."""
    _fields_ = [("item_work", ctypes.c_int), ("wide_min", ctypes.c_int), ("wg_per_cu", ctypes.c_int),
                ("max_split", ctypes.c_int)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)
_V = ctypes.c_void_p
_i, _d = ctypes.c_int, ctypes.c_double

_SIGS = {
    "g6_open": (_i, [_i]),
    "g6_close": (_i, [_i]),
    "g6_npipes": (_i, []),
    "g6_set_tunit": (None, [_i]),
    "g6_set_xunit": (None, [_i]),
    "g6_set_j_particle": (_i, [_i, _i, _i, _d, _d, _d, _D, _D, _D, _D, _D]),
    "g6mi_set_j_particles": (_i, [_i, _i, _I, _I, _D, _D, _D, _D, _D, _D, _D]),
    "g6_set_ti": (None, [_i, _d]),
    "g6calc_firsthalf": (_i, [_i, _i, _i, _I, _D, _D, _D, _D, _D, _d, _D]),
    "g6calc_lasthalf": (_i, [_i, _i, _i, _I, _D, _D, _d, _D, _D, _D, _D]),
    "g6calc_lasthalf2": (_i, [_i, _i, _i, _I, _D, _D, _d, _D, _D, _D, _D, _I]),
    "g6_nearest_neighbour": (_i, [_i, _i, _I, _D]),
    "g6_read_neighbour_list": (_i, [_i]),
    "g6_get_neighbour_list": (_i, [_i, _i, _i, _I, _I]),
    "g6mi_last_error": (ctypes.c_char_p, [_i]),
    "g6mi_nb_max": (_i, []),
    "g6mi_set_precision": (_i, [_i, _i]),
    "g6mi_get_precision": (_i, [_i]),
    "g6mi_set_neighbour_lists": (_i, [_i, _i]),
    "g6mi_set_shape": (_i, [_i, _i, _i]),
    "g6mi_set_spatial": (_i, [_i, _i]),
    "g6mi_set_fused_predict": (_i, [_i, _i]),
    "g6mi_get_shape": (_i, [_i, _I]),
    "g6mi_enable_timing": (_i, [_i, _i]),
    "g6mi_last_timing": (_i, [_i, _D]),
    "g6mi_timing_totals": (_i, [_i, _D, _I]),
    "g6mi_set_j_particles_device": (_i, [_i, _i, _V, _V, _V, _V, _V, _V, _V, _V]),
    "g6mi_calc_device": (_i, [_i, _i, _i, _V, _V, _V, _d, _V, _V, _V, _V, _V, _V, _V]),
    "g6mi_calc_device_noalloc": (_i, [_i, _i, _i, _V, _V, _V, _d, _V, _V, _V, _V, _V, _V, _V]),
    "g6mi_device_info": (_i, [_i, _I]),
    "g6mi_last_status": (_i, [_i, _I]),
    "g6mi_batch_calc": (_i, [_i, _i, _V, _i, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
    "g6mi_batch_calc_device": (_i, [_i, _i, _V, _i, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V]),
    "g6mi_batch_use_graph": (_i, [_i, _i]),
    "g6mi_batch_set_tuning": (_i, [_i, ctypes.POINTER(BatchTuning)]),
    "g6mi_batch_get_tuning": (_i, [_i, ctypes.POINTER(BatchTuning)]),
    "g6mi_batch_autotune": (_i, [_i, _i, _V, _i, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V, ctypes.c_char_p, _i,
                                 ctypes.POINTER(BatchTuning)]),
    "g6mi_hermite_init": (_i, [_i, _i, _d, _d, _d, _d, _d, _d]),
    "g6mi_hermite_advance": (_i, [_i, _d, ctypes.c_longlong, _D, ctypes.POINTER(ctypes.c_longlong)]),
    "g6mi_hermite_state": (_i, [_i, _i, _D, _D, _D, _D, _D, _D, _D]),
}
EXPORTED = tuple(_SIGS)


def _L():
    """The loaded libg6mi.so with its signatures declared."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: PyTorch ships its own libamdhip64 with
        # the same soname as /opt/rocm's.  Whichever is loaded first serves
        # both, so load torch's first; torch's device pointers and streams
        # are then valid in this library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_0902_4463_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            try:
                f = getattr(lib, name)
            except AttributeError as e:
                raise ImportError(f"{LIB_PATH} lacks {name}: rebuild it") from e
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class G6Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return None if a is None else a.ctypes.data_as(_D)


def _pi(a):
    return None if a is None else a.ctypes.data_as(_I)


def _ptr(t):
    """Device address of a torch tensor (or an int address, or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def last_error(id: int) -> str:
    msg = _L().g6mi_last_error(id)
    return msg.decode() if msg else ""


def check(id: int, rc: int, allow_warn: bool = True) -> int:
    if rc < 0 or (rc > 0 and not allow_warn):
        raise G6Error(rc, last_error(id))
    return rc


# ------------------------------------------------ GRAPE-6 calling sequence

def g6_open(id: int) -> int:
    return _L().g6_open(id)


def g6_close(id: int) -> int:
    return _L().g6_close(id)


def g6_npipes() -> int:
    return _L().g6_npipes()


def g6_set_tunit(v: int) -> None:
    _L().g6_set_tunit(v)


def g6_set_xunit(v: int) -> None:
    _L().g6_set_xunit(v)


def g6_set_j_particle(id, address, index, tj, dtj, mass, k18, j6, a2, v, x) -> int:
    k18, j6, a2, v, x = (_f64(q, (3,)) for q in (k18, j6, a2, v, x))
    return _L().g6_set_j_particle(id, int(address), int(index), float(tj), float(dtj),
                                  float(mass), _pd(k18), _pd(j6), _pd(a2), _pd(v), _pd(x))


def g6mi_set_j_particles(id, n, address, index, tj, dtj, mass, j6, a2, v, x) -> int:
    """Bulk g6_set_j_particle: n records from arrays (vectors as (n, 3))."""
    address, index = _i32(address), _i32(index)
    tj, mass = _f64(tj, (n,)), _f64(mass, (n,))
    j6, a2, v, x = (_f64(q, (n, 3)) for q in (j6, a2, v, x))
    dtj = None if dtj is None else _f64(dtj, (n,))
    return _L().g6mi_set_j_particles(id, int(n), _pi(address), _pi(index), _pd(tj), _pd(dtj), _pd(mass),
                                     _pd(j6), _pd(a2), _pd(v), _pd(x))


def g6_set_ti(id: int, ti: float) -> None:
    _L().g6_set_ti(id, float(ti))


def g6calc_firsthalf(id, nj, ni, index, xi, vi, aold, j6old, phiold, eps2, h2) -> int:
    index = _i32(index)
    xi, vi = _f64(xi, (ni, 3)), _f64(vi, (ni, 3))
    h2 = None if h2 is None else _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (ni,)))
    aold = None if aold is None else _f64(aold, (ni, 3))
    j6old = None if j6old is None else _f64(j6old, (ni, 3))
    phiold = None if phiold is None else _f64(phiold, (ni,))
    return _L().g6calc_firsthalf(id, nj, ni, _pi(index), _pd(xi), _pd(vi), _pd(aold),
                                 _pd(j6old), _pd(phiold), float(eps2), _pd(h2))


def g6calc_lasthalf(id, nj, ni, index, xi, vi, eps2, h2, acc, jerk, pot) -> int:
    """acc, jerk ((ni, 3) float64) and pot ((ni,) float64) are written in place."""
    index = _i32(index)
    return _L().g6calc_lasthalf(id, nj, ni, _pi(index), None, None, float(eps2), None,
                                _pd(acc), _pd(jerk), _pd(pot))


def g6calc_lasthalf2(id, nj, ni, index, xi, vi, eps2, h2, acc, jerk, pot, nnbindex) -> int:
    index = _i32(index)
    return _L().g6calc_lasthalf2(id, nj, ni, _pi(index), None, None, float(eps2), None,
                                 _pd(acc), _pd(jerk), _pd(pot), _pi(nnbindex))


def g6_nearest_neighbour(id, ni, nnbindex, r2nn) -> int:
    return _L().g6_nearest_neighbour(id, ni, _pi(nnbindex), _pd(r2nn))


def g6_read_neighbour_list(id) -> int:
    return _L().g6_read_neighbour_list(id)


def g6_get_neighbour_list(id, ipipe, maxlength, nblen, nbl) -> int:
    """nblen: int32 array of length >= 1; nbl: int32 array of length maxlength."""
    return _L().g6_get_neighbour_list(id, ipipe, maxlength, _pi(nblen), _pi(nbl))


# ------------------------------------------------------------- extensions

def g6mi_last_error(id: int) -> str:
    return last_error(id)


def g6mi_nb_max() -> int:
    return _L().g6mi_nb_max()


def g6mi_set_precision(id, prec) -> int:
    if isinstance(prec, str):
        prec = PRECISIONS[prec]
    return _L().g6mi_set_precision(id, prec)


def g6mi_get_precision(id) -> int:
    return _L().g6mi_get_precision(id)


def g6mi_set_neighbour_lists(id, on) -> int:
    return _L().g6mi_set_neighbour_lists(id, int(bool(on)))


def g6mi_set_spatial(id, mode) -> int:
    """0 off, 1 double-single blocks of at least 65536 (default), 2 every double-single calculation."""
    return _L().g6mi_set_spatial(id, int(mode))


def g6mi_set_fused_predict(id, on) -> int:
    """1: one-block calls predict their j-tiles inside the interaction kernel."""
    return _L().g6mi_set_fused_predict(id, int(bool(on)))


def g6mi_set_shape(id, i_per_group, j_splits) -> int:
    return _L().g6mi_set_shape(id, int(i_per_group), int(j_splits))


def g6mi_get_shape(id):
    out = np.zeros(4, dtype=np.int32)
    check(id, _L().g6mi_get_shape(id, _pi(out)))
    return dict(i_per_group=int(out[0]), j_splits=int(out[1]), j_tile=int(out[2]),
                workgroups=int(out[3]))


def g6mi_enable_timing(id, on) -> int:
    return _L().g6mi_enable_timing(id, int(bool(on)))


def g6mi_last_timing(id):
    ms = np.zeros(3)
    check(id, _L().g6mi_last_timing(id, _pd(ms)))
    return dict(predict_ms=float(ms[0]), force_ms=float(ms[1]), reduce_ms=float(ms[2]))


def g6mi_timing_totals(id):
    ms = np.zeros(3)
    cnt = np.zeros(1, dtype=np.int32)
    check(id, _L().g6mi_timing_totals(id, _pd(ms), _pi(cnt)))
    return dict(predict_ms=float(ms[0]), force_ms=float(ms[1]), reduce_ms=float(ms[2]), count=int(cnt[0]))


def g6mi_set_j_particles_device(id, nj, t, mass, index, x, v, a2, j6, stream=None) -> int:
    return _L().g6mi_set_j_particles_device(id, int(nj), _ptr(t), _ptr(mass), _ptr(index),
                                            _ptr(x), _ptr(v), _ptr(a2), _ptr(j6), _stream(stream))


def g6mi_calc_device(id, nj, ni, islot, xi, vi, eps2, h2, acc, jerk, pot, nnb=None, r2nn=None,
                     stream=None) -> int:
    return _L().g6mi_calc_device(id, int(nj), int(ni), _ptr(islot), _ptr(xi), _ptr(vi),
                                 float(eps2), _ptr(h2), _ptr(acc), _ptr(jerk), _ptr(pot),
                                 _ptr(nnb), _ptr(r2nn), _stream(stream))


def g6mi_calc_device_noalloc(id, nj, ni, islot, xi, vi, eps2, h2, acc, jerk, pot, nnb=None, r2nn=None,
                             stream=None) -> int:
    """g6mi_calc_device with its work buffers in the library's static
    per-GPU scratch array (no allocation)."""
    return _L().g6mi_calc_device_noalloc(id, int(nj), int(ni), _ptr(islot), _ptr(xi), _ptr(vi),
                                         float(eps2), _ptr(h2), _ptr(acc), _ptr(jerk), _ptr(pot),
                                         _ptr(nnb), _ptr(r2nn), _stream(stream))


def g6mi_device_info(id):
    out = np.zeros(2, dtype=np.int32)
    check(id, _L().g6mi_device_info(id, _pi(out)))
    return dict(compute_units=int(out[0]), clock_mhz=int(out[1]))


def g6mi_last_status(id) -> int:
    """Status flags of the last calculation (FLAG_* bits)."""
    out = np.zeros(1, dtype=np.int32)
    check(id, _L().g6mi_last_status(id, _pi(out)))
    return int(out[0])


# ------------------------------------------------------------ batched calls

def clusters(joff, nj, ioff, ni, ti, eps2) -> np.ndarray:
    """Cluster descriptors (struct g6mi_cluster) from per-cluster sequences."""
    n = len(joff)
    out = np.zeros(n, dtype=CLUSTER_DTYPE)
    out["joff"], out["nj"], out["ioff"], out["ni"] = joff, nj, ioff, ni
    out["ti"], out["eps2"] = ti, eps2
    return out


def _cl_host(cl):
    cl = np.ascontiguousarray(cl, dtype=CLUSTER_DTYPE)
    return cl, cl.ctypes.data


def g6mi_batch_calc(id, cl, ni_total, islot, xi, vi, h2, acc, jerk, pot, nnb=None, r2nn=None,
                    stream=None) -> int:
    """cl: host descriptors (CLUSTER_DTYPE array); the rest device buffers."""
    cl, addr = _cl_host(cl)
    return _L().g6mi_batch_calc(id, len(cl), addr, int(ni_total), _ptr(islot), _ptr(xi), _ptr(vi), _ptr(h2),
                                _ptr(acc), _ptr(jerk), _ptr(pot), _ptr(nnb), _ptr(r2nn), _stream(stream))


def g6mi_batch_calc_device(id, ncl, d_cl, ni_total, islot, xi, vi, h2, acc, jerk, pot, nnb=None, r2nn=None,
                           stream=None) -> int:
    """d_cl: device buffer holding ncl descriptors (32 bytes each)."""
    return _L().g6mi_batch_calc_device(id, int(ncl), _ptr(d_cl), int(ni_total), _ptr(islot), _ptr(xi),
                                       _ptr(vi), _ptr(h2), _ptr(acc), _ptr(jerk), _ptr(pot), _ptr(nnb),
                                       _ptr(r2nn), _stream(stream))


def g6mi_batch_use_graph(id, on) -> int:
    return _L().g6mi_batch_use_graph(id, int(bool(on)))


def g6mi_batch_set_tuning(id, tuning=None) -> int:
    """tuning: dict with item_work, wide_min, wg_per_cu, max_split, or None
    for the defaults."""
    if tuning is None:
        return _L().g6mi_batch_set_tuning(id, None)
    t = BatchTuning(**{k: int(v) for k, v in tuning.items()})
    return _L().g6mi_batch_set_tuning(id, ctypes.byref(t))


def g6mi_batch_get_tuning(id) -> dict:
    t = BatchTuning()
    check(id, _L().g6mi_batch_get_tuning(id, ctypes.byref(t)))
    return t.as_dict()


def g6mi_batch_autotune(id, cl, ni_total, islot, xi, vi, h2, acc, jerk, pot, nnb=None, r2nn=None,
                        stream=None, cache_path=None, reps=3):
    """Returns (rc, chosen tuning as a dict)."""
    cl, addr = _cl_host(cl)
    t = BatchTuning()
    path = None if cache_path is None else os.fsencode(cache_path)
    rc = _L().g6mi_batch_autotune(id, len(cl), addr, int(ni_total), _ptr(islot), _ptr(xi), _ptr(vi),
                                  _ptr(h2), _ptr(acc), _ptr(jerk), _ptr(pot), _ptr(nnb), _ptr(r2nn),
                                  _stream(stream), path, int(reps), ctypes.byref(t))
    return rc, t.as_dict()


# ------------------------------------------------ device-resident block steps

def g6mi_hermite_init(id, n, eps2, h2, eta, eta_s, dt_max, dt_min) -> int:
    return _L().g6mi_hermite_init(id, int(n), float(eps2), float(h2), float(eta), float(eta_s), float(dt_max),
                                  float(dt_min))


def g6mi_hermite_advance(id, t_end, max_steps):
    """Returns (rc, time reached, block steps, particle steps)."""
    t = np.zeros(1)
    cnt = (ctypes.c_longlong * 2)()
    rc = _L().g6mi_hermite_advance(id, float(t_end), int(max_steps), _pd(t), cnt)
    return rc, float(t[0]), int(cnt[0]), int(cnt[1])


def g6mi_hermite_state(id, n):
    """State of slots 0..n-1 as a dict of arrays (x, v, acc, jerk, pot, t, dt)."""
    out = dict(x=np.zeros((n, 3)), v=np.zeros((n, 3)), acc=np.zeros((n, 3)), jerk=np.zeros((n, 3)),
               pot=np.zeros(n), t=np.zeros(n), dt=np.zeros(n))
    check(id, _L().g6mi_hermite_state(id, int(n), *(_pd(out[k]) for k in ("x", "v", "acc", "jerk", "pot", "t", "dt"))))
    return out


# --------------------------------------------------- convenience wrappers

class Session:
    """A GRAPE-6 handle driven through the calls above (argument marshalling
    only): load a j-memory, run one block's force calculation, read the
    results back."""

    def __init__(self, id: int = 0, precision: str = "ds", neighbour_lists: bool = True):
        self.id = id
        check(id, g6_open(id))
        check(id, g6mi_set_precision(id, precision))
        check(id, g6mi_set_neighbour_lists(id, neighbour_lists))

    def close(self):
        g6_close(self.id)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load(self, jm) -> None:
        """Store every slot of a ``workloads.JMemory`` (bulk g6_set_j_particle)."""
        check(self.id, g6mi_set_j_particles(self.id, jm.n, np.arange(jm.n), jm.index, jm.t, None, jm.m,
                                            jm.j6, jm.a2, jm.v, jm.x))

    def calc(self, nj, ti, index, xi, vi, eps2, h2, neighbours=True):
        ni = len(index)
        g6_set_ti(self.id, ti)
        check(self.id, g6calc_firsthalf(self.id, nj, ni, index, xi, vi, None, None, None, eps2, h2))
        acc = np.zeros((ni, 3)); jerk = np.zeros((ni, 3)); pot = np.zeros(ni)
        nnb = np.zeros(ni, dtype=np.int32)
        rc = check(self.id, g6calc_lasthalf2(self.id, nj, ni, index, xi, vi, eps2, h2, acc, jerk, pot, nnb))
        r2nn = np.zeros(ni)
        nn_idx = np.zeros(ni, dtype=np.int32)
        check(self.id, g6_nearest_neighbour(self.id, ni, nn_idx, r2nn))
        out = dict(acc=acc, jerk=jerk, pot=pot, nn_index=nnb, nn_r2=r2nn, nonfinite=rc == WARN)
        if neighbours:
            out["nb_overflow"] = check(self.id, g6_read_neighbour_list(self.id)) == WARN
            counts = np.zeros(ni, dtype=np.int64)
            lists = np.full((ni, NB_MAX), -1, dtype=np.int32)
            ln = np.zeros(1, dtype=np.int32)
            for i in range(ni):
                buf = np.zeros(NB_MAX, dtype=np.int32)
                check(self.id, g6_get_neighbour_list(self.id, i, NB_MAX, ln, buf))
                counts[i] = ln[0]
                k = min(int(ln[0]), NB_MAX)
                lists[i, :k] = buf[:k]
            out["nb_count"], out["nb_list"] = counts, lists
        return out
