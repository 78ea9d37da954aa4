"""The float32 bounds that let the grouped interaction paths skip per-pair
neighbour work, checked by replaying the kernels' float32 steps in numpy.

1. Group neighbour flags.  The grouped paths keep, per group, the minimum of
   the softened r^2 + eps2 (formed as one fma chain seeded with eps2) and flag
   the group when it is below (h^2 + eps2)(1 + 2^-20); the exact test of a
   flagged group's records uses r^2 = fma(dz, dz, fma(dy, dy, dx * dx)) < h^2.
   Every pair that the exact test takes must lie in a flagged group.
2. Quiet far tiles.  A far tile skips its nearest-neighbour and flag work
   when the least softened r^2 any of its records can give,
   ((|x_i - c| - r_t)^+)^2 + eps2 with margins of 2^-18, exceeds what the
   search and the flags need; that least value must never exceed a value the
   far path computes for a record of the tile.
3. Seeded searches.  The search starts below the softened r^2 to a nearby
   record, computed with the double-single separation of Eq. (3), times
   1 + 2^-16, plus the least normal float32; the far path's value for the
   same pair must stay below that seed, also at distance zero.

fma is replayed as the float64 product and sum of float32 operands rounded
to float32 (the product is exact; a double rounding moves the result by at
most one float32 unit, far inside every margin checked here).
"""

import numpy as np
import pytest

from tests.test_far_tile_bound import ds_split, is_far, ibox, rel_to_centre, tile_info, threshold_draw

F32, F64 = np.float32, np.float64
FLAG = F32(1.0 + 2.0 ** -20)
QLO, QHI = F32(1.0 - 2.0 ** -18), F32(1.0 + 2.0 ** -18)
SEED = F32(1.0 + 2.0 ** -16)
TINY = F32(2.0 ** -126)


def fma32(a, b, c):
    return (np.asarray(a, F32).astype(F64) * np.asarray(b, F32).astype(F64) + np.asarray(c, F32).astype(F64)).astype(F32)


def r2_exact_test(d):
    """r^2 as the exact neighbour test forms it."""
    return fma32(d[..., 2], d[..., 2], fma32(d[..., 1], d[..., 1], (d[..., 0] * d[..., 0]).astype(F32)))


def softened(d, eps2):
    """r^2 + eps2 as the grouped paths form it."""
    e = F32(eps2)
    return fma32(d[..., 2], d[..., 2], fma32(d[..., 1], d[..., 1], fma32(d[..., 0], d[..., 0], e)))


def flag_bound(h2, eps2):
    return (F32(F32(h2) + F32(eps2)) * FLAG).astype(F32)


@pytest.mark.parametrize("eps2", [0.0, 1e-8, (1 / 64) ** 2, 1e-4, 1.0])
@pytest.mark.parametrize("h2", [1e-6, 1e-4, 0.05, 1.0])
def test_flag_bound_covers_every_exact_neighbour(h2, eps2):
    rng = np.random.default_rng(int(1e6 * h2) + int(1e8 * eps2))
    n = 200000
    # separations on and around the neighbour sphere, and well inside it
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    r = np.sqrt(h2) * np.where(rng.random(n) < 0.9, 1.0 + rng.uniform(-3e-6, 3e-6, n), rng.random(n))
    # the same separation at several magnitudes of the coordinates' exponents
    d = (u * r[:, None]).astype(F32)
    inside = r2_exact_test(d) < F32(h2)
    assert inside.sum() > 1000
    s = softened(d, eps2)
    assert np.all(s[inside] < flag_bound(h2, eps2)), (h2, eps2)


def test_flag_bound_needs_its_margin():
    """Without the factor 1 + 2^-20 some exact neighbours near the sphere fall
    outside the flag (r^2 + eps2 rounds up to (h^2 + eps2) or beyond), so the
    margin is not decoration."""
    rng = np.random.default_rng(3)
    missed = 0
    for eps2, h2 in ((1e-4, 1e-4), ((1 / 64) ** 2, 1e-4), (1.0, 0.05)):
        u = rng.normal(size=(200000, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        d = (u * (np.sqrt(h2) * (1 - rng.uniform(0, 1e-6, 200000)))[:, None]).astype(F32)
        inside = r2_exact_test(d) < F32(h2)
        missed += int(np.sum(softened(d, eps2)[inside] >= F32(F32(h2) + F32(eps2))))
    assert missed > 0


def least_softened(b, rt, eps2):
    """The kernel's least softened r^2 for a particle at b (float32, relative
    to the tile centre) against a tile of radius bound rt."""
    dc = np.sqrt(fma32(b[..., 2], b[..., 2], fma32(b[..., 1], b[..., 1], (b[..., 0] * b[..., 0]).astype(F32))))
    gap = np.maximum((dc * QLO).astype(F32) - (F32(rt) * QHI).astype(F32), F32(0.0)).astype(F32)
    return (fma32(gap, gap, eps2) * QLO).astype(F32)


K_FAR = 0.75  # the library's far criterion (G6MI_FAR_K)


def far_pairs(xj, xi, k=K_FAR):
    """For a tile (xj) and an i-block (xi) that the kernel takes as far: the
    far path's softened-r^2 inputs (d per pair), the particles relative to
    the centre and the radius bound; None if the tile is not far."""
    jh, jl = ds_split(xj)
    ih, il = ds_split(xi)
    chi, clo, rt, blo, bhi = tile_info(jh, jl)
    ilo, ihi = ibox(ih, il)
    if not is_far(blo, bhi, ilo, ihi, rt, k):
        return None
    a = rel_to_centre(jh, jl, chi, clo)
    b = rel_to_centre(ih, il, chi, clo)
    d = (a[None, :, :] - b[:, None, :]).astype(F32)
    return d, b, rt, (jh, jl, ih, il)


@pytest.mark.parametrize("eps2", [0.0, 1e-8, 1e-4])
def test_quiet_tile_bound_is_below_every_far_value(eps2):
    rng = np.random.default_rng(11 + int(1e8 * eps2))
    tiles = 0
    slack = []
    for t in range(300):
        s = 10.0 ** rng.uniform(-4, -1)
        xj, xi = threshold_draw(rng, K_FAR, rng.choice([0.0, 0.01, 0.3, 1e4]), s)
        if t % 3 == 0:  # i-particles farther out as well
            xi = xi + (xi - xj.mean(axis=0)) * rng.uniform(0, 20)
        got = far_pairs(xj, xi)
        if got is None:
            continue
        d, b, rt, _ = got
        tiles += 1
        s_far = softened(d, eps2)                       # [ni, nj]
        least = least_softened(b, rt, eps2)             # [ni]
        assert np.all(least[:, None] <= s_far), (t, float(np.min(s_far - least[:, None])))
        slack.append(float(np.min(s_far / np.maximum(least[:, None], 1e-38))))
    assert tiles >= 100, tiles
    # the bound is not vacuous: at the threshold it comes within a factor of a few
    assert min(slack) < 4.0


@pytest.mark.parametrize("eps2", [0.0, 1e-8, 1e-4])
def test_seed_stays_above_the_far_path_value(eps2):
    """The seed is formed from the Eq. (3) separation in float32; for every
    pair that a far tile could hold, the far path's softened r^2 is below it."""
    rng = np.random.default_rng(21 + int(1e8 * eps2))
    tiles = 0
    for t in range(200):
        s = 10.0 ** rng.uniform(-4, -1)
        xj, xi = threshold_draw(rng, K_FAR, rng.choice([0.0, 0.01, 0.3, 1e4]), s)
        got = far_pairs(xj, xi)
        if got is None:
            continue
        d, _, _, (jh, jl, ih, il) = got
        tiles += 1
        d3 = ((jh[None] - ih[:, None]).astype(F32) + (jl[None] - il[:, None]).astype(F32)).astype(F32)
        seed = fma32(softened(d3, eps2), SEED, TINY)
        assert np.all(softened(d, eps2) < seed), t
    assert tiles >= 60, tiles


def test_seed_at_distance_zero():
    """Coincident particles at eps = 0: both paths give exactly zero, and the
    seed (the least normal float32 above it) still lets the search take the
    pair."""
    x = np.array([[0.3, -0.2, 1e4]])
    h, l = ds_split(x)
    d3 = ((h - h) + (l - l)).astype(F32)
    s = softened(d3[None], 0.0)
    assert s[0, 0] == 0.0
    seed = fma32(s, SEED, TINY)
    assert s[0, 0] < seed[0, 0]
    # without the added constant the strict search test would never take it
    assert not (s[0, 0] < (s * SEED).astype(F32)[0, 0])
