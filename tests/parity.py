"""Comparison of GPU results with the float64 oracle.

Acceptance per i-particle (relative errors with vector 2-norms):
  acceleration  |da| <= TOL_ACC  |a|
  jerk          |dj| <= TOL_JERK |j|
  potential     |dphi| <= TOL_POT |phi|
A particle whose sum cancels strongly -- conditioning kappa = sum_k |a_ik| /
|a_i| above 10 -- may instead satisfy |da| <= TOL |a| kappa / 10; such
particles are counted and reported, never hidden.  Potentials have kappa = 1
(all terms share a sign).

Nearest neighbour: accepted when the index equals the oracle's, or when the
float64 squared distance to the GPU's choice is within a factor (1 + 1e-6)
of the oracle's minimum.  Neighbour list: accepted when every index in the
symmetric difference with the oracle's list lies within 1e-6 h^2 of the
neighbour sphere.
"""

from __future__ import annotations

import numpy as np

TOL_ACC = 2e-6
TOL_JERK = 1e-5
TOL_POT = 1e-6
TIE_REL = 1e-6
KAPPA_FREE = 10.0


def rel_errors(gpu, ref):
    ea = np.linalg.norm(gpu["acc"] - ref["acc"], axis=1) / np.maximum(np.linalg.norm(ref["acc"], axis=1), 1e-300)
    ej = np.linalg.norm(gpu["jerk"] - ref["jerk"], axis=1) / np.maximum(np.linalg.norm(ref["jerk"], axis=1), 1e-300)
    ep = np.abs(gpu["pot"] - ref["pot"]) / np.maximum(np.abs(ref["pot"]), 1e-300)
    return ea, ej, ep


def force_report(gpu, ref, tol_acc=TOL_ACC, tol_jerk=TOL_JERK, tol_pot=TOL_POT):
    """Error statistics and the pass/fail decision of the acceptance rule.
    ``ref`` must hold acc_abs / jerk_abs (oracle run with conditioning)."""
    ea, ej, ep = rel_errors(gpu, ref)
    ka = ref["acc_abs"] / np.maximum(np.linalg.norm(ref["acc"], axis=1), 1e-300)
    kj = ref["jerk_abs"] / np.maximum(np.linalg.norm(ref["jerk"], axis=1), 1e-300)
    ok_a = (ea <= tol_acc) | ((ka > KAPPA_FREE) & (ea <= tol_acc * ka / KAPPA_FREE))
    ok_j = (ej <= tol_jerk) | ((kj > KAPPA_FREE) & (ej <= tol_jerk * kj / KAPPA_FREE))
    ok_p = ep <= tol_pot
    return dict(
        n=int(ea.size),
        acc_max=float(ea.max(initial=0)), jerk_max=float(ej.max(initial=0)), pot_max=float(ep.max(initial=0)),
        acc_p999=float(np.percentile(ea, 99.9)) if ea.size else 0.0,
        jerk_p999=float(np.percentile(ej, 99.9)) if ej.size else 0.0,
        acc_conditioned=int(np.sum(ok_a & (ea > tol_acc))), jerk_conditioned=int(np.sum(ok_j & (ej > tol_jerk))),
        acc_fail=int(np.sum(~ok_a)), jerk_fail=int(np.sum(~ok_j)), pot_fail=int(np.sum(~ok_p)),
        ok=bool(ok_a.all() and ok_j.all() and ok_p.all()),
        worst_acc=int(np.argmax(ea)) if ea.size else -1,
    )


def r2_to(xj, jindex, xi, i_rows, chosen):
    """float64 squared distance from i-particle rows to the j-particles with
    the given particle indices (chosen == -1 gives +inf)."""
    pos = {int(k): n for n, k in enumerate(jindex)}
    out = np.full(len(i_rows), np.inf)
    for q, (r, c) in enumerate(zip(i_rows, chosen)):
        if c >= 0:
            d = xj[pos[int(c)]] - xi[r]
            out[q] = float(d @ d)
    return out


def nn_report(gpu_idx, ref_idx, ref_r2, xj, jindex, xi):
    gpu_idx = np.asarray(gpu_idx)
    ref_idx = np.asarray(ref_idx)
    diff = np.nonzero(gpu_idx != ref_idx)[0]
    r2g = r2_to(xj, jindex, xi, diff, gpu_idx[diff])
    tie = r2g <= ref_r2[diff] * (1 + TIE_REL)
    return dict(mismatch=int(diff.size), ties=int(tie.sum()), fail=int((~tie).sum()), ok=bool(tie.all()))


def nb_report(gpu_count, gpu_list, ref_count, ref_list, xj, jindex, xi, h2, cap=256):
    """Compare neighbour lists (rows of particle indices, -1 padded)."""
    pos = {int(k): n for n, k in enumerate(jindex)}
    h2 = np.broadcast_to(np.asarray(h2, dtype=np.float64), (len(gpu_count),))
    bad = 0
    ties = 0
    overflow_rows = 0
    for i in range(len(gpu_count)):
        gc, rc = int(gpu_count[i]), int(ref_count[i])
        if rc > cap or gc > cap:
            overflow_rows += 1
            continue
        g = set(int(v) for v in gpu_list[i, :min(gc, cap)])
        r = set(int(v) for v in ref_list[i, :min(rc, cap)])
        if list(gpu_list[i, :min(gc, cap)]) != sorted(g):
            bad += 1
            continue
        for k in g ^ r:
            d = xj[pos[k]] - xi[i]
            if abs(float(d @ d) - h2[i]) <= TIE_REL * h2[i]:
                ties += 1
            else:
                bad += 1
    return dict(fail=bad, ties=ties, overflow_rows=overflow_rows, ok=bad == 0)
