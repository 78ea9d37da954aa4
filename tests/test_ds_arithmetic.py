"""Double-single (DS) claims of the paper, checked with numpy float32.

These tests document what the DS position format and the separation of
Eq. (3) deliver, independently of any GPU code: a DS number is the pair
hi = fl32(x), lo = fl32(x - hi); the separation of two DS numbers is
(x_j,hi - x_i,hi) + (x_j,lo - x_i,lo), evaluated in float32.
"""

import json
import os

import numpy as np

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def ds_split(x):
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    lo = (x - hi.astype(np.float64)).astype(np.float32)
    return hi, lo


def ds_sep(xj, xi):
    """Eq. (3), Sec. 2.3, in float32 (three operations)."""
    jh, jl = ds_split(xj)
    ih, il = ds_split(xi)
    return (jh - ih) + (jl - il)


def test_split_round_trip_is_48_bit():
    """Sec. 2.2 footnote: DS carries 48 mantissa bits."""
    bits = GOLDEN["ds_mantissa_bits"]["value"]
    rng = np.random.default_rng(1)
    x = rng.normal(size=100000) * 10.0 ** rng.uniform(-6, 6, 100000)
    hi, lo = ds_split(x)
    err = np.abs(x - (hi.astype(np.float64) + lo.astype(np.float64)))
    assert np.all(err <= 2.0 ** -bits * np.abs(x))


def test_separation_resolution_one_part_in_1e7():
    """Sec. 2.3: Eq. (3) resolves separations to one part in 1e7 or better,
    whereas a plain float32 difference of close positions does not."""
    res = GOLDEN["ds_separation_resolution"]["value"]
    rng = np.random.default_rng(2)
    xi = rng.uniform(-10, 10, 200000)
    sep = 10.0 ** rng.uniform(-6, -1, xi.size) * rng.choice([-1, 1], xi.size)
    xj = xi + sep
    exact = xj - xi  # float64 reference of the same two float64 positions
    ds = ds_sep(xj, xi).astype(np.float64)
    rel = np.abs(ds - exact) / np.abs(exact)
    # the float32 result is rounded twice (hi-difference sum, then storage),
    # so "one part in 1e7" holds up to 2^-23 = 1.19e-7 in the worst case
    assert np.max(rel) <= 2.0 ** -23
    assert np.percentile(rel, 99.9) <= res
    sp = (xj.astype(np.float32) - xi.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(sp - exact) / np.abs(exact)) > 100 * res


def test_four_digit_example():
    """Sec. 2.3: two positions agreeing in their first four significant
    digits keep about three significant digits in a float32 difference and
    (at least) seven after Eq. (3), where the float32 result is the limit."""
    g = GOLDEN["four_digit_example"]
    xi = 1234.56789012345
    xj = 1234.98765432109
    exact = xj - xi
    sp = float(np.float32(xj) - np.float32(xi))
    ds = float(ds_sep(np.array([xj]), np.array([xi]))[0])
    sp_digits = -np.log10(abs(sp - exact) / abs(exact))
    ds_digits = -np.log10(abs(ds - exact) / abs(exact) + 1e-300)
    assert sp_digits < g["sp_digits"] + 1.5
    assert ds_digits >= g["stored_digits"]


def test_flop_convention_constants():
    assert GOLDEN["flops_per_interaction"]["value"] == 60
    # each of the three coordinate subtractions (1 flop) becomes Eq. (3) (3 flops)
    assert GOLDEN["flops_per_interaction_ds"]["value"] == 60 + 3 * (GOLDEN["ds_difference_flops"]["value"] - 1)
