"""Seeded particle distributions for the force-evaluation workloads.

Every generator takes either a seed or a ``numpy.random.Generator`` (PCG64)
and works in float64.  Units are Henon N-body units (G = M = 1, virial
radius 1, E = -1/4 for the Plummer model), the units the paper's test runs
use (Sec. 3: equal-mass Plummer spheres integrated for fractions of an
N-body time unit).

Nothing here evaluates a force, a potential or a predictor: the arrays are
plain samples of the distributions named below.
"""

from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

# Henon-unit scale of the Plummer model: virial radius 1 for G = M = 1.
PLUMMER_LENGTH = 3.0 * np.pi / 16.0


def _rng(seed_or_rng) -> np.random.Generator:
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.Generator(np.random.PCG64(int(seed_or_rng)))


def _isotropic(rng: np.random.Generator, radius: np.ndarray) -> np.ndarray:
    """Vectors of the given length with uniformly random direction."""
    n = radius.shape[0]
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    out = np.empty((n, 3))
    out[:, 0] = radius * s * np.cos(phi)
    out[:, 1] = radius * s * np.sin(phi)
    out[:, 2] = radius * z
    return out


def plummer(n: int, seed_or_rng, masses: np.ndarray | None = None):
    """Plummer sphere by the Aarseth-Henon-Wielen (1974) recipe.

    Radii come from inverting the cumulative mass profile (mass fractions
    above 0.999 are rejected, which truncates the infinite model); speeds
    are drawn by von Neumann rejection from the isotropic distribution
    function, g(q) = q^2 (1 - q^2)^{7/2} with q = v / v_escape.  The system
    is moved to its centre-of-mass frame and scaled to Henon units
    (lengths times 3*pi/16, velocities divided by sqrt(3*pi/16)).

    Returns (x, v), each (n, 3) float64.
    """
    rng = _rng(seed_or_rng)
    if n <= 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    # radii
    radii = np.empty(0)
    while radii.size < n:
        x1 = rng.uniform(0.0, 1.0, 2 * (n - radii.size) + 16)
        x1 = x1[(x1 > 0.0) & (x1 <= 0.999)]
        radii = np.concatenate([radii, (x1 ** (-2.0 / 3.0) - 1.0) ** -0.5])
    r = radii[:n]
    x = _isotropic(rng, r)
    # speeds: rejection sampling of q in [0, 1) under g(q) <= 0.1
    q = np.empty(0)
    while q.size < n:
        m = 4 * (n - q.size) + 16
        cand = rng.uniform(0.0, 1.0, m)
        y = rng.uniform(0.0, 0.1, m)
        keep = y < cand * cand * (1.0 - cand * cand) ** 3.5
        q = np.concatenate([q, cand[keep]])
    q = q[:n]
    vesc = np.sqrt(2.0) * (1.0 + r * r) ** -0.25
    v = _isotropic(rng, q * vesc)
    w = np.full(n, 1.0 / n) if masses is None else np.asarray(masses, dtype=np.float64)
    wsum = w.sum()
    x -= (w[:, None] * x).sum(axis=0) / wsum
    v -= (w[:, None] * v).sum(axis=0) / wsum
    x *= PLUMMER_LENGTH
    v /= np.sqrt(PLUMMER_LENGTH)
    return x, v


def salpeter_masses(n: int, seed_or_rng, slope: float = -2.35,
                    m_lo: float = 0.1, m_hi: float = 100.0) -> np.ndarray:
    """Power-law IMF dN/dm ~ m^slope on [m_lo, m_hi] by inverse transform,
    renormalised so that the total mass is 1."""
    rng = _rng(seed_or_rng)
    p = slope + 1.0  # -1.35 for Salpeter
    u = rng.uniform(0.0, 1.0, n)
    m = (m_lo ** p + u * (m_hi ** p - m_lo ** p)) ** (1.0 / p)
    return m / m.sum()


def _solve_kepler(mean_anom: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly E from M = E - e sin E by Newton iteration."""
    ecc = np.where(e > 0.8, np.pi * np.ones_like(mean_anom), mean_anom)
    for _ in range(100):
        f = ecc - e * np.sin(ecc) - mean_anom
        d = 1.0 - e * np.cos(ecc)
        step = f / d
        ecc = ecc - step
        if np.max(np.abs(step)) < 1e-15:
            break
    return ecc


def hard_binaries(centres_x, centres_v, m1, m2, seed_or_rng,
                  a_lo=1e-5, a_hi=1e-3):
    """Replace each centre by a Keplerian binary of masses (m1, m2).

    Semi-major axis log-uniform in [a_lo, a_hi], thermal eccentricity
    (e = sqrt(U)), isotropic orbital orientation and uniform mean anomaly.
    Returns positions and velocities of both members, (2B, 3) each, with
    members 2b and 2b+1 belonging to binary b, plus the drawn (a, e).
    """
    rng = _rng(seed_or_rng)
    cx = np.asarray(centres_x, dtype=np.float64)
    cv = np.asarray(centres_v, dtype=np.float64)
    nb = cx.shape[0]
    a = np.exp(rng.uniform(np.log(a_lo), np.log(a_hi), nb))
    e = np.sqrt(rng.uniform(0.0, 1.0, nb))
    mean_anom = rng.uniform(0.0, 2.0 * np.pi, nb)
    ecc_anom = _solve_kepler(mean_anom, e)
    # orbital frame basis: P along pericentre, Q in-plane perpendicular
    pvec = _isotropic(rng, np.ones(nb))
    t = _isotropic(rng, np.ones(nb))
    qvec = t - (t * pvec).sum(axis=1, keepdims=True) * pvec
    qvec /= np.linalg.norm(qvec, axis=1, keepdims=True)
    mtot = m1 + m2
    cos_e, sin_e = np.cos(ecc_anom), np.sin(ecc_anom)
    sq = np.sqrt(1.0 - e * e)
    rel_x = (a * (cos_e - e))[:, None] * pvec + (a * sq * sin_e)[:, None] * qvec
    nmot = np.sqrt(mtot / a ** 3)
    fac = nmot * a / (1.0 - e * cos_e)
    rel_v = (-fac * sin_e)[:, None] * pvec + (fac * sq * cos_e)[:, None] * qvec
    x = np.empty((2 * nb, 3))
    v = np.empty((2 * nb, 3))
    x[0::2] = cx - (m2 / mtot) * rel_x
    x[1::2] = cx + (m1 / mtot) * rel_x
    v[0::2] = cv - (m2 / mtot) * rel_v
    v[1::2] = cv + (m1 / mtot) * rel_v
    return x, v, a, e


def synthetic_derivatives(n: int, seed_or_rng, a_scale: float = 1.0,
                          j_scale: float = 3.0):
    """Stand-in Taylor coefficients a/2 and jerk/6 for the j-predictor.

    Gaussian vectors whose magnitudes match those of a Plummer sphere in
    Henon units (|a| ~ 1, |jerk| ~ 3).  They only serve as input to the
    prediction polynomial; they are not forces of the sampled system."""
    rng = _rng(seed_or_rng)
    a = rng.normal(0.0, a_scale / np.sqrt(3.0), (n, 3))
    j = rng.normal(0.0, j_scale / np.sqrt(3.0), (n, 3))
    return a / 2.0, j / 6.0


@dataclass
class JMemory:
    """One GRAPE-style j-particle memory, slot k = row k.

    ``a2`` holds a/2 and ``j6`` holds jerk/6 (the pre-scaled Taylor
    coefficients a GRAPE-6 client stores), ``t`` the time of each
    particle's last correction."""

    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    index: np.ndarray
    t: np.ndarray
    a2: np.ndarray
    j6: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.m.shape[0])


def make_jmemory(x, v, m, index=None, t=None, a2=None, j6=None, meta=None) -> JMemory:
    n = np.asarray(m).shape[0]
    return JMemory(
        x=np.ascontiguousarray(x, dtype=np.float64).reshape(n, 3),
        v=np.ascontiguousarray(v, dtype=np.float64).reshape(n, 3),
        m=np.ascontiguousarray(m, dtype=np.float64).reshape(n),
        index=np.ascontiguousarray(np.arange(n) if index is None else index, dtype=np.int32),
        t=np.zeros(n) if t is None else np.ascontiguousarray(t, dtype=np.float64),
        a2=np.zeros((n, 3)) if a2 is None else np.ascontiguousarray(a2, dtype=np.float64),
        j6=np.zeros((n, 3)) if j6 is None else np.ascontiguousarray(j6, dtype=np.float64),
        meta=dict(meta or {}),
    )


def active_set(n: int, count: int, seed: int) -> np.ndarray:
    """The first ``count`` entries of a seeded permutation of range(n)."""
    rng = _rng(seed)
    return np.sort(rng.permutation(n)[:count]).astype(np.int32)


# ---------------------------------------------------------------------------
# The concrete workloads.  Sizes, softening and neighbour radii follow the
# evaluation recipe: Plummer spheres in Henon units (Sec. 3), Salpeter masses
# for the throughput sweep, hard binaries for the precision stress case.
# ---------------------------------------------------------------------------

def config_c1(seed: int = 1) -> JMemory:
    """Equal-mass Plummer N=1024, eps = 1/64, neighbour radius 0.1, all
    particles at t = 0 with zero Taylor coefficients (the start of a run)."""
    n = 1024
    rng = _rng(seed)
    x, v = plummer(n, rng)
    return make_jmemory(x, v, np.full(n, 1.0 / n), meta=dict(
        name="plummer_N1024_eps1/64", eps2=2.0 ** -12, h2=0.1 ** 2, ti=0.0, seed=seed))


def config_c2(seed: int = 2, n: int = 32768) -> JMemory:
    """Equal-mass Plummer N=32768, eps = 1e-4 (initial conditions)."""
    rng = _rng(seed)
    x, v = plummer(n, rng)
    return make_jmemory(x, v, np.full(n, 1.0 / n), meta=dict(
        name=f"plummer_N{n}_eps1e-4", eps2=1e-8, h2=1e-4, ti=0.0, seed=seed))


def config_c3(seed: int = 3, n: int = 2 ** 20) -> JMemory:
    """Throughput workload: Plummer N=2^20, Salpeter masses (0.1-100,
    slope -2.35, total mass 1), eps = 1e-4, neighbour radius 0.01.  All
    particles were last corrected at t = 0 and are predicted to t = 2^-10
    with stand-in Taylor coefficients."""
    rng = _rng(seed)
    m = salpeter_masses(n, rng)
    x, v = plummer(n, rng, masses=m)
    a2, j6 = synthetic_derivatives(n, rng)
    return make_jmemory(x, v, m, a2=a2, j6=j6, meta=dict(
        name=f"plummer_salpeter_N{n}_eps1e-4", eps2=1e-8, h2=1e-4,
        ti=2.0 ** -10, seed=seed))


def config_c5(seed: int = 5, n: int = 2 ** 18, binary_fraction: float = 0.05,
              shift: float = 1e4) -> JMemory:
    """Precision stress: equal-mass Plummer N=2^18 in which 5% of the
    particles are members of hard binaries (B = round(0.025 N) binaries,
    a log-uniform in [1e-5, 1e-3], thermal e), the whole system translated
    by (1e4, 1e4, 1e4), eps = 0, neighbour radius 0.01."""
    rng = _rng(seed)
    nbin = int(round(0.5 * binary_fraction * n))
    ncent = n - nbin
    xc, vc = plummer(ncent, rng)
    mass = 1.0 / n
    bx, bv, a, e = hard_binaries(xc[:nbin], vc[:nbin], mass, mass, rng)
    x = np.concatenate([bx, xc[nbin:]]) + shift
    v = np.concatenate([bv, vc[nbin:]])
    is_bin = np.zeros(n, dtype=bool)
    is_bin[: 2 * nbin] = True
    return make_jmemory(x, v, np.full(n, mass), meta=dict(
        name=f"plummer_binaries_N{n}_shift{shift:g}", eps2=0.0, h2=1e-4, ti=0.0,
        seed=seed, n_binaries=nbin, binary_a=a, binary_e=e, is_binary=is_bin))


def random_cluster(n: int, seed: int, ti: float = 2.0 ** -6,
                   mass_kind: str = "salpeter", shift: float = 0.0) -> JMemory:
    """Small mixed test system: Plummer positions, Salpeter or equal masses,
    last-correction times on a power-of-two grid below ``ti`` and stand-in
    Taylor coefficients, so that the predictor does non-trivial work."""
    rng = _rng(seed)
    m = salpeter_masses(n, rng) if mass_kind == "salpeter" else np.full(n, 1.0 / max(n, 1))
    x, v = plummer(n, rng, masses=m if n else None)
    a2, j6 = synthetic_derivatives(n, rng)
    # block-step times: t_k = ti - dt_k * u with dt_k a power of two
    dt = 2.0 ** -rng.integers(6, 12, n)
    t = ti - dt * rng.integers(0, 2, n)
    return make_jmemory(x + shift, v, m, t=t, a2=a2, j6=j6, meta=dict(
        name=f"random_cluster_N{n}_seed{seed}", ti=ti, seed=seed))


@dataclass
class ClusterBatch:
    """Independent clusters concatenated in one j-memory: cluster c owns
    slots joff[c] .. joff[c+1]-1; its active i-particles are the slots in
    active[ioff[c] .. ioff[c+1]-1]; ti[c] and eps2[c] are its own prediction
    time and softening."""

    jm: JMemory
    joff: np.ndarray
    ioff: np.ndarray
    active: np.ndarray
    ti: np.ndarray
    eps2: np.ndarray
    h2: np.ndarray

    @property
    def nclusters(self) -> int:
        return int(self.joff.shape[0] - 1)


def config_c4(seed: int = 4, nclusters: int = 256, n_lo: int = 256, n_hi: int = 8192) -> ClusterBatch:
    """Batched workload: independent Plummer clusters with N log-uniform in
    [n_lo, n_hi], Salpeter masses (each cluster's total mass 1), centres
    offset uniformly in [-100, 100]^3, individual block times (power-of-two
    steps below each cluster's own time) and their own active blocks (2^k
    particles, k uniform in 0 .. log2 N).  Softening 1e-4 for every cluster,
    neighbour radius 0.01."""
    rng = _rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), nclusters)).astype(np.int64)
    joff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    ntot = int(joff[-1])
    x = np.empty((ntot, 3)); v = np.empty((ntot, 3)); m = np.empty(ntot)
    t = np.empty(ntot); a2 = np.empty((ntot, 3)); j6 = np.empty((ntot, 3))
    ti = np.empty(nclusters)
    active = []
    ioff = [0]
    for c in range(nclusters):
        n = int(sizes[c]); lo, hi = int(joff[c]), int(joff[c + 1])
        mc = salpeter_masses(n, rng)
        xc, vc = plummer(n, rng, masses=mc)
        x[lo:hi] = xc + rng.uniform(-100.0, 100.0, 3)
        v[lo:hi] = vc
        m[lo:hi] = mc
        ti[c] = rng.integers(1, 64) * 2.0 ** -8
        dt = 2.0 ** -rng.integers(6, 12, n)
        t[lo:hi] = ti[c] - dt * rng.integers(0, 2, n)
        ac, jc = synthetic_derivatives(n, rng)
        a2[lo:hi], j6[lo:hi] = ac, jc
        k = int(rng.integers(0, int(np.log2(n)) + 1))
        act = np.sort(rng.permutation(n)[: 2 ** k]) + lo
        active.append(act)
        ioff.append(ioff[-1] + len(act))
    jm = make_jmemory(x, v, m, t=t, a2=a2, j6=j6, meta=dict(name=f"clusters{nclusters}_N{n_lo}-{n_hi}", seed=seed))
    return ClusterBatch(jm=jm, joff=joff, ioff=np.array(ioff, dtype=np.int64),
                        active=np.concatenate(active).astype(np.int32), ti=ti,
                        eps2=np.full(nclusters, 1e-8), h2=np.full(nclusters, 1e-4))


def input_digest(*arrays) -> str:
    """sha256 over the raw bytes of the given arrays (logged with results)."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
