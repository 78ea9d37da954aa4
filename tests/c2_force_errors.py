"""Config 2 (equal-mass Plummer N = 32768, eps = 1e-4, eta = 0.01) to t = 1
through the host-side Hermite driver on libg6mi (a GPU is required), every
block step's forces compared with the float64 oracle on the same predicted
state: all i-particles of a block up to `--cap`, else a seeded sample of that
many.  Not a pytest module (it runs for minutes); it prints progress to
stderr and one JSON line with the per-step error record summarised:

    python tests/c2_force_errors.py --precision ds --cap 1024 > c2_errors_ds.json
"""

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
from hermite import BlockStepIntegrator, HermiteState  # noqa: E402
from tests.hermite_oracle import Shadowed  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--precision", choices=["ds", "fp32", "fp64"], default="ds")
    ap.add_argument("--cap", type=int, default=1024)
    ap.add_argument("--t-end", type=float, default=1.0)
    ap.add_argument("--dump", default=None, help="npz file for the inputs of the first failing calls")
    args = ap.parse_args(argv)
    jm = workloads.config_c2()
    eps2 = jm.meta["eps2"]
    st = HermiteState(jm.x, jm.v, jm.m)
    b = Shadowed(jm.n, eps2, args.precision, cap=args.cap)
    b.keep_fail_inputs = args.dump is not None
    w0 = time.perf_counter()
    try:
        it = BlockStepIntegrator(st, b, eta=0.01, dt_max=2.0 ** -4)
        e0 = st.energies()[2]
        marks = []
        k = 1
        while k / 64 <= args.t_end + 1e-12:
            it.run(k / 64)
            if k % 8 == 0:
                marks.append(dict(t=k / 64, dE_over_E=(st.energies()[2] - e0) / e0))
            print(f"[c2 errors {args.precision}] t={it.time:.4f} block steps={it.steps} worst={b.worst} "
                  f"fails={len(b.fails)} {time.perf_counter() - w0:.0f} s", file=sys.stderr, flush=True)
            k += 1
    finally:
        b.close()
    if args.dump and b.fail_inputs:
        np.savez_compressed(args.dump, eps2=eps2, **{f"{k}_{q}": v for q, d in enumerate(b.fail_inputs)
                                                     for k, v in d.items()})
    rec = np.array([r[1:] for r in b.record], dtype=float)
    ni, checked, acc, jerk, pot, cond = rec.T
    out = dict(config="c2", n=jm.n, precision=args.precision, eta=0.01, t_end=args.t_end, cap=args.cap,
               block_steps=it.steps, particle_steps=it.particle_steps, force_calls=len(b.record),
               particles_checked=int(checked.sum()), fails=len(b.fails),
               worst=dict(acc=float(acc.max()), jerk=float(jerk.max()), pot=float(pot.max())),
               p99=dict(acc=float(np.percentile(acc, 99)), jerk=float(np.percentile(jerk, 99)),
                        pot=float(np.percentile(pot, 99))),
               conditioned=int(cond.sum()), energy=marks, wall_s=round(time.perf_counter() - w0, 1),
               first_fails=[(t, n, {k: r[k] for k in ("acc_max", "jerk_max", "pot_max")}) for t, n, r in b.fails[:3]])
    print(json.dumps(out), flush=True)
    return 0 if not b.fails else 1


if __name__ == "__main__":
    sys.exit(main())
