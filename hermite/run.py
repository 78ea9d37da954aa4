"""Run a Hermite block-step integration on libg6mi and print one JSON line.

    python -m hermite.run --config c1 --precision ds
    python -m hermite.run --config c2 --precision fp64 --t-end 1
    python -m hermite.run --config c2 --device          # block steps on the GPU

Configurations (seeded, see ``workloads``): c1 = equal-mass Plummer N=1024,
eps = 1/64, to t = 1/8; c2 = equal-mass Plummer N=32768, eps = 1e-4, to t = 1.
Both use eta = 0.01 (Aarseth criterion).  Reported: relative energy error
dE/E at every multiple of 1/8 (the accuracy measure of Sec. 3.2), number of
block steps, particle steps, the block-size histogram (Sec. 3.1, Fig. block)
and the time spent in the library and in the host-side integrator.

--device runs the same integrator inside the library (g6mi_hermite_*: every
block step a replayed graph of kernels, the host only reading the state at
the reporting times); the block-size histogram is then not available.
"""

from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from hermite.driver import BlockStepIntegrator, G6Backend, HermiteState  # noqa: E402


class TimedBackend:
    def __init__(self, inner):
        self.inner = inner
        self.seconds = 0.0
        self.calls = 0

    def set_j(self, st, sel):
        t0 = time.perf_counter()
        self.inner.set_j(st, sel)
        self.seconds += time.perf_counter() - t0

    def force(self, ti, index, xi, vi):
        t0 = time.perf_counter()
        out = self.inner.force(ti, index, xi, vi)
        self.seconds += time.perf_counter() - t0
        self.calls += 1
        return out


def energies(m, v, pot):
    kin = 0.5 * float(np.sum(m * np.sum(v * v, axis=1)))
    return kin + 0.5 * float(np.sum(m * pot))


def run_device(args, jm, t_end, dt_max, marks):
    """The integrator inside the library: state read back at each mark."""
    import paper_0902_4463_amd as g6
    hid = 0
    g6.check(hid, g6.g6_open(hid))
    g6.check(hid, g6.g6mi_set_precision(hid, args.precision))
    g6.check(hid, g6.g6mi_set_neighbour_lists(hid, False))
    if args.batch_tuning:
        iw, wm, wg, ms = (int(x) for x in args.batch_tuning.split(","))
        g6.check(hid, g6.g6mi_batch_set_tuning(hid, dict(item_work=iw, wide_min=wm, wg_per_cu=wg, max_split=ms)))
    g6.check(hid, g6.g6mi_set_j_particles(hid, jm.n, np.arange(jm.n), jm.index, np.zeros(jm.n), None, jm.m,
                                          np.zeros((jm.n, 3)), np.zeros((jm.n, 3)), jm.v, jm.x))
    w0 = time.perf_counter()
    g6.check(hid, g6.g6mi_hermite_init(hid, jm.n, jm.meta["eps2"], 0.0, args.eta, 0.01, dt_max, 2.0 ** -40),
             allow_warn=False)
    st = g6.g6mi_hermite_state(hid, jm.n)
    e0 = energies(jm.m, st["v"], st["pot"])
    out = []
    steps = (0, 0)
    for mark in marks:
        rc, t, bsteps, psteps = g6.g6mi_hermite_advance(hid, mark, 1 << 40)
        g6.check(hid, rc, allow_warn=False)
        st = g6.g6mi_hermite_state(hid, jm.n)
        assert np.all(st["t"] == mark), "particles not synchronised at the mark"
        out.append(dict(t=t, dE_over_E=(energies(jm.m, st["v"], st["pot"]) - e0) / e0))
        steps = (bsteps, psteps)
        print(f"[hermite/device] t={t:.4f} dE/E={out[-1]['dE_over_E']:.3e} steps={bsteps}", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - w0
    g6.g6_close(hid)
    return out, steps, wall


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=["c1", "c2"], default="c1")
    ap.add_argument("--precision", choices=["ds", "fp32", "fp64"], default="ds")
    ap.add_argument("--eta", type=float, default=0.01)
    ap.add_argument("--t-end", type=float, default=None)
    ap.add_argument("--device", action="store_true", help="block steps inside the library, on the GPU")
    ap.add_argument("--batch-tuning", default=None,
                    help="item_work,wide_min,wg_per_cu,max_split of the force launches of --device runs")
    args = ap.parse_args(argv)
    jm = workloads.config_c1() if args.config == "c1" else workloads.config_c2()
    t_end = args.t_end if args.t_end is not None else (0.125 if args.config == "c1" else 1.0)
    dt_max = 0.125 if args.config == "c1" else 2.0 ** -4
    if args.device:
        marks = [0.125 * (k + 1) for k in range(int(round(t_end / 0.125)))]
        energy, (bsteps, psteps), wall = run_device(args, jm, t_end, dt_max, marks)
        print(json.dumps(dict(
            config=args.config, n=jm.n, precision=args.precision, eta=args.eta, eps2=jm.meta["eps2"],
            mode="device", t_end=energy[-1]["t"] if energy else 0.0, energy=energy, block_steps=bsteps,
            particle_steps=psteps, mean_block=psteps / max(1, bsteps), wall_s=round(wall, 2),
            pairs=float(psteps) * jm.n)), flush=True)
        return
    st = HermiteState(jm.x, jm.v, jm.m)
    backend = TimedBackend(G6Backend(jm.n, jm.meta["eps2"], precision=args.precision))
    w0 = time.perf_counter()
    it = BlockStepIntegrator(st, backend, eta=args.eta, dt_max=dt_max)
    e0 = st.energies()[2]
    energies = []
    mark = 0.125
    while it.time < t_end:
        it.step()
        if it.time >= mark and it.synchronised():
            energies.append(dict(t=it.time, dE_over_E=(st.energies()[2] - e0) / e0))
            print(f"[hermite] t={it.time:.4f} dE/E={energies[-1]['dE_over_E']:.3e} steps={it.steps}",
                  file=sys.stderr, flush=True)
            mark += 0.125
    wall = time.perf_counter() - w0
    backend.inner.close()
    hist = collections.Counter(int(np.log2(s.n_active)) for s in it.log)
    print(json.dumps(dict(
        config=args.config, n=jm.n, precision=args.precision, eta=args.eta, eps2=jm.meta["eps2"],
        t_end=it.time, energy=energies, block_steps=it.steps, particle_steps=it.particle_steps,
        mean_block=it.particle_steps / max(1, it.steps),
        log2_block_histogram=dict(sorted(hist.items())),
        wall_s=round(wall, 2), library_s=round(backend.seconds, 2), force_calls=backend.calls,
        pairs=float(it.particle_steps) * jm.n)), flush=True)


if __name__ == "__main__":
    main()
