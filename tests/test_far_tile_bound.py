"""Error bound of the far-tile separation in the spatially ordered
double-single kernel, checked by replaying its float32/float64 steps in numpy.

For a tile of double-single j-records whose box lies at least K tile radii
from a workgroup's i-box, the kernel forms A = x_j - c and B = x_i - c (c the
tile centre) in float64 from the exact sums hi + lo, rounds each once to
float32, and takes the pair separation d = fl32(A' - B').  The stated bound
is |d - D| <= 2 (1 + 1/K) u |D| with u = 2^-24 and D = x_j - x_i of the
double-single positions, against 2 u |D| for Eq. (3) of Sec. 2.3.  Every step
below mirrors the kernel: the DS split, the outward-rounded boxes, the
centre and radius of the tile, the float32 far criterion and the separation.
"""

import zlib

import numpy as np
import pytest

F32, F64 = np.float32, np.float64
U = 2.0 ** -24


def ds_split(x):
    x = np.asarray(x, dtype=F64)
    hi = x.astype(F32)
    lo = (x - hi.astype(F64)).astype(F32)
    return hi, lo


def outward(hi, lo):
    """float32 bounds down <= hi + lo <= up (hi + lo exact in float64)."""
    v = hi.astype(F64) + lo.astype(F64)
    f = v.astype(F32)
    down = np.where(f.astype(F64) > v, np.nextafter(f, F32(-np.inf)), f)
    up = np.where(f.astype(F64) < v, np.nextafter(f, F32(np.inf)), f)
    return down, up


def tile_info(xh, xl):
    """Centre (DS), radius and box of one tile, as the tile-table kernel."""
    down, up = outward(xh, xl)
    blo, bhi = down.min(axis=0), up.max(axis=0)
    c = 0.5 * (blo.astype(F64) + bhi.astype(F64))
    chi, clo = ds_split(c)
    a = (xh.astype(F64) + xl.astype(F64)) - (chi.astype(F64) + clo.astype(F64))
    r = np.sqrt(np.max(np.sum(a * a, axis=1)))
    rt = F32(F32(r) * F32(1.0 + 2.0 ** -20))
    return chi, clo, rt, blo, bhi


def ibox(xh, xl):
    down, up = outward(xh, xl)
    return down.min(axis=0), up.max(axis=0)


def is_far(blo, bhi, ilo, ihi, rt, k):
    g2 = F32(0.0)
    for d in range(3):
        gd = max(F32(0.0), max(F32(blo[d] - ihi[d]), F32(ilo[d] - bhi[d])))
        g2 = F32(g2 + F32(gd * gd))
    reach = F32(F32(k) * rt)
    return bool(g2 >= F32(reach * reach))


def rel_to_centre(xh, xl, chi, clo):
    c64 = chi.astype(F64) + clo.astype(F64)
    return ((xh.astype(F64) + xl.astype(F64)) - c64).astype(F32)


def far_errors(xj, xi, k, centring=None):
    """Relative separation errors |d - D| / (u |D|) of every pair of one
    tile (xj) with an i-block (xi), or None if the kernel would not take the
    tile as far; also checks |x_j - c| <= r_t."""
    jh, jl = ds_split(xj)
    ih, il = ds_split(xi)
    chi, clo, rt, blo, bhi = tile_info(jh, jl)
    a64 = (jh.astype(F64) + jl.astype(F64)) - (chi.astype(F64) + clo.astype(F64))
    assert np.all(np.sqrt(np.sum(a64 * a64, axis=1)) <= rt)
    ilo, ihi = ibox(ih, il)
    if not is_far(blo, bhi, ilo, ihi, rt, k):
        return None
    centring = centring or rel_to_centre
    a = centring(jh, jl, chi, clo)
    b = centring(ih, il, chi, clo)
    d = (a[None, :, :] - b[:, None, :]).astype(F64)          # float32 difference
    xj_ds = jh.astype(F64) + jl.astype(F64)
    xi_ds = ih.astype(F64) + il.astype(F64)
    exact = xj_ds[None, :, :] - xi_ds[:, None, :]
    err = np.linalg.norm(d - exact, axis=2)
    return err / (U * np.linalg.norm(exact, axis=2))


def eq3_errors(xj, xi):
    jh, jl = ds_split(xj)
    ih, il = ds_split(xi)
    d = ((jh[None] - ih[:, None]) + (jl[None] - il[:, None])).astype(F64)
    exact = (jh.astype(F64) + jl.astype(F64))[None] - (ih.astype(F64) + il.astype(F64))[:, None]
    return np.linalg.norm(d - exact, axis=2) / (U * np.linalg.norm(exact, axis=2))


def draw(rng, origin, tile_size, gap_over_r, k, ntile=256, ni=64):
    """A tile of ntile records in a cube of side tile_size around a point
    near `origin`, and an i-block of ni particles whose nearest point sits
    about gap_over_r * K tile radii away along a random direction."""
    p = origin + rng.uniform(-1, 1, 3) * tile_size
    xj = p + rng.uniform(-0.5, 0.5, (ntile, 3)) * tile_size
    r_est = 0.5 * np.sqrt(3.0) * tile_size
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    isize = tile_size * 10.0 ** rng.uniform(-2, 1)
    q = p + u * (r_est * (k * gap_over_r + np.sqrt(3.0)) + np.sqrt(3.0) * isize)
    xi = q + rng.uniform(-0.5, 0.5, (ni, 3)) * isize
    return xj, xi


SCENARIOS = [
    ("unit sphere", 0.0, (-4, -1)),
    ("translated by 1e4", 1e4, (-3, 0)),
    ("centre near 0.01, i near 0.5", 0.01, (-4, -2)),
    ("straddling the origin", 0.0, (-1, 0)),
]


@pytest.mark.parametrize("k", [0.75, 1.0, 2.0])
@pytest.mark.parametrize("name,origin,log_size", SCENARIOS)
def test_far_separation_within_bound(name, origin, log_size, k):
    rng = np.random.default_rng(zlib.crc32(f"{name} {k}".encode()))
    bound = 2.0 * (1.0 + 1.0 / k)
    worst, tiles = 0.0, 0
    for t in range(60):
        size = 10.0 ** rng.uniform(*log_size)
        gap = 1.0 + 10.0 ** rng.uniform(-6, 0.5) if t % 2 else 1.0 + 1e-4
        xj, xi = draw(rng, origin, size, gap, k)
        e = far_errors(xj, xi, k)
        if e is None:
            continue
        tiles += 1
        worst = max(worst, float(e.max()))
        assert e.max() <= bound * (1.0 + 1e-6), (name, t, float(e.max()))
    assert tiles >= 20, tiles  # the draws do exercise far tiles
    print(f"{name} K={k}: worst |d-D|/(u|D|) = {worst:.3f} (bound {bound}) over {tiles} far tiles")


def test_advisor_case_and_eq3_reference():
    """A tile centred near 0.01 and i-particles near 0.5 (where x_i - c is
    not within a factor of two of x_i, so a float32 hi/lo difference rounds
    twice): the far path stays within 4 u |D| at K = 1, and Eq. (3) within
    2 u |D|."""
    rng = np.random.default_rng(7)
    xj = 0.01 + rng.uniform(-0.5, 0.5, (256, 3)) * 1e-4
    xi = 0.5 + rng.uniform(-0.5, 0.5, (512, 3)) * 1e-2
    e = far_errors(xj, xi, 1.0)
    assert e is not None and e.max() <= 4.0 * (1 + 1e-6)
    assert eq3_errors(xj, xi).max() <= 2.0 * (1 + 1e-6)


def test_near_tile_is_not_far():
    """An i-block overlapping the tile's box never takes the far path."""
    rng = np.random.default_rng(9)
    xj = rng.uniform(-0.5, 0.5, (256, 3)) * 1e-2
    xi = rng.uniform(-0.5, 0.5, (64, 3)) * 1e-2
    assert far_errors(xj, xi, 1.0) is None


def threshold_draw(rng, k, origin, s):
    """Records on a shell of radius ~s and i-particles just past K tile
    radii from the tile's box along an axis: the near-side records then have
    |A| ~ r_t, |D| ~ K r_t and |B| ~ (1 + K) r_t, where the bound is tight."""
    p = origin + rng.uniform(-1, 1, 3) * s * 3
    d = rng.normal(size=(256, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    xj = p + d * s * rng.uniform(0.9, 1, (256, 1))
    xi = np.repeat(p[None], 256, 0)
    xi[:, rng.integers(3)] += rng.choice([-1, 1]) * (s + k * s * np.sqrt(3) * 1.0001)
    xi += rng.uniform(-1, 1, (256, 3)) * s * 1e-3
    return xj, xi


def test_threshold_tiles_and_float32_centring():
    """Tiles at the far threshold (K = 1) over several origins: the kernel's
    float64 centring stays within 2 (1 + 1/K) = 4; forming x - c as
    (x_hi - c_hi) + (x_lo - c_lo) in float32 instead rounds twice on each
    side and leaves that bound on the same draws."""
    def f32_centring(xh, xl, chi, clo):
        return ((xh - chi) + (xl - clo)).astype(F32)

    def worst(form):
        rng = np.random.default_rng(1)
        w, n = 0.0, 0
        for _ in range(400):
            s = 10.0 ** rng.uniform(-4, -1)
            xj, xi = threshold_draw(rng, 1.0, rng.choice([0.0, 0.01, 0.3, 1e4]), s)
            e = far_errors(xj, xi, 1.0, form)
            if e is not None:
                n += 1
                w = max(w, float(e.max()))
        return w, n

    w_kernel, n = worst(rel_to_centre)
    assert n >= 300
    assert w_kernel <= 4.0 * (1 + 1e-6), w_kernel
    w_f32, _ = worst(f32_centring)
    assert w_f32 > 4.0, w_f32


def test_threshold_tiles_at_the_default_criterion():
    """The library's far criterion, K = 0.75 (G6MI_FAR_K): tiles just past
    the threshold over several origins stay within 2 (1 + 1/K) = 4.67
    float32 roundings."""
    rng = np.random.default_rng(5)
    k = 0.75
    worst, n = 0.0, 0
    for _ in range(400):
        s = 10.0 ** rng.uniform(-4, -1)
        xj, xi = threshold_draw(rng, k, rng.choice([0.0, 0.01, 0.3, 1e4]), s)
        e = far_errors(xj, xi, k)
        if e is not None:
            n += 1
            worst = max(worst, float(e.max()))
    assert n >= 300, n
    assert worst <= 2.0 * (1.0 + 1.0 / k) * (1 + 1e-6), worst
    print(f"K=0.75 threshold tiles: worst |d-D|/(u|D|) = {worst:.3f} over {n} far tiles")
