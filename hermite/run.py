"""Run a Hermite block-step integration on libg6mi and print one JSON line.

    python -m hermite.run --config c1 --precision ds
    python -m hermite.run --config c2 --precision fp64 --t-end 1

Configurations (seeded, see ``workloads``): c1 = equal-mass Plummer N=1024,
eps = 1/64, to t = 1/8; c2 = equal-mass Plummer N=32768, eps = 1e-4, to t = 1.
Both use eta = 0.01 (Aarseth criterion).  Reported: relative energy error
dE/E at every multiple of 1/8 (the accuracy measure of Sec. 3.2), number of
block steps, particle steps, the block-size histogram (Sec. 3.1, Fig. block)
and the time spent in the library and in the host-side integrator.
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", choices=["c1", "c2"], default="c1")
    ap.add_argument("--precision", choices=["ds", "fp32", "fp64"], default="ds")
    ap.add_argument("--eta", type=float, default=0.01)
    ap.add_argument("--t-end", type=float, default=None)
    args = ap.parse_args(argv)
    jm = workloads.config_c1() if args.config == "c1" else workloads.config_c2()
    t_end = args.t_end if args.t_end is not None else (0.125 if args.config == "c1" else 1.0)
    dt_max = 0.125 if args.config == "c1" else 2.0 ** -4
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
