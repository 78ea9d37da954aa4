"""Accuracy study: relative energy error against the time-step parameter eta
for each precision variant of the force kernel, and the mean block size
against N (the paper's accuracy and block-size measurements, Sec. 3.2,
Fig. devseta and Fig. block), with the block steps run inside the library
(g6mi_hermite_*).

    python -m hermite.study --n 32768 131072 --eta 1e-4 3e-4 1e-3 3e-3 0.01 0.03 0.1 0.3 \\
        --precision ds fp64 --t-end 0.25 > study.jsonl

Each run: equal-mass Plummer sphere (seeded, Henon units), softening 1e-4,
4th-order Hermite with Aarseth steps (first step min(eta, 0.01) |a|/|jerk|),
dt_max 2^-4, from t = 0 to t_end; the energy is read at every multiple of
1/8 (all particles synchronised there).  A run stops early, marked
"capped", after max_steps block steps: with float32 forces and small eta the
third derivative of the corrector drowns in force rounding, the steps
collapse, and the run would not finish.  One JSON line per run.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402


def energy(m, v, pot):
    return 0.5 * float(np.sum(m * np.sum(v * v, axis=1))) + 0.5 * float(np.sum(m * pot))


def run_one(g6, hid, jm, eta, prec, t_end, dt_max, max_steps):
    n = jm.n
    g6.check(hid, g6.g6_open(hid))
    try:
        g6.check(hid, g6.g6mi_set_precision(hid, prec))
        g6.check(hid, g6.g6mi_set_neighbour_lists(hid, False))
        g6.check(hid, g6.g6mi_set_j_particles(hid, n, np.arange(n), jm.index, np.zeros(n), None, jm.m,
                                              np.zeros((n, 3)), np.zeros((n, 3)), jm.v, jm.x))
        w0 = time.perf_counter()
        rc = g6.g6mi_hermite_init(hid, n, jm.meta["eps2"], 0.0, eta, min(eta, 0.01), dt_max, 2.0 ** -40)
        g6.check(hid, rc)
        st = g6.g6mi_hermite_state(hid, n)
        e0 = energy(jm.m, st["v"], st["pot"])
        marks, t, steps, psteps, capped = [], 0.0, 0, 0, False
        k = 1
        while k * 0.125 <= t_end + 1e-12 and not capped:
            mark = k * 0.125
            # advance in eighths of the interval, reporting each one reached
            for q in range(1, 9):
                sub = mark - 0.125 + q * 0.125 / 8
                rc, t, steps, psteps = g6.g6mi_hermite_advance(hid, sub, max(0, max_steps - steps))
                g6.check(hid, rc)
                if t < sub:
                    capped = True
                    break
                print(f"[study]   N={n} eta={eta} {prec} reached t={sub:.5f} blocks={steps}", file=sys.stderr,
                      flush=True)
            if capped:
                break
            st = g6.g6mi_hermite_state(hid, n)
            marks.append(dict(t=mark, dE_over_E=(energy(jm.m, st["v"], st["pot"]) - e0) / e0))
            print(f"[study]   N={n} eta={eta} {prec} t={mark}: dE/E={marks[-1]['dE_over_E']:.3e} blocks={steps}",
                  file=sys.stderr, flush=True)
            k += 1
        wall = time.perf_counter() - w0
        return dict(n=n, eta=eta, precision=prec, eps2=jm.meta["eps2"], t_end=t_end, t_reached=t, capped=capped,
                    energy=marks, block_steps=steps, particle_steps=psteps,
                    mean_block=psteps / max(1, steps), pairs=float(psteps) * n, wall_s=round(wall, 2))
    finally:
        g6.g6_close(hid)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, nargs="+", default=[32768, 131072])
    ap.add_argument("--eta", type=float, nargs="+", default=[1e-4, 3e-4, 1e-3, 3e-3, 0.01, 0.03, 0.1, 0.3])
    ap.add_argument("--precision", nargs="+", default=["ds", "fp64"], choices=["ds", "fp32", "fp64"])
    ap.add_argument("--t-end", type=float, default=0.25)
    ap.add_argument("--dt-max", type=float, default=2.0 ** -4)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--seed", type=int, default=2)
    args = ap.parse_args(argv)
    import paper_0902_4463_amd as g6
    for n in args.n:
        jm = workloads.config_c2(seed=args.seed, n=n)
        for eta in args.eta:
            for prec in args.precision:
                r = run_one(g6, 0, jm, eta, prec, args.t_end, args.dt_max, args.max_steps)
                print(json.dumps(r), flush=True)
                last = r["energy"][-1]["dE_over_E"] if r["energy"] else float("nan")
                print(f"[study] N={n} eta={eta} {prec}: dE/E={last:.3e} blocks={r['block_steps']} "
                      f"mean block={r['mean_block']:.1f} {r['wall_s']} s{' CAPPED' if r['capped'] else ''}",
                      file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
