"""Properties of the seeded synthetic inputs (no force arithmetic)."""

import numpy as np
import pytest

import workloads
from workloads.generators import PLUMMER_LENGTH


def test_plummer_seeded_and_centred():
    x1, v1 = workloads.plummer(4096, 7)
    x2, v2 = workloads.plummer(4096, 7)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
    assert np.allclose(x1.mean(axis=0), 0, atol=1e-14)
    assert np.allclose(v1.mean(axis=0), 0, atol=1e-14)


def test_plummer_half_mass_radius_and_kinetic_energy():
    """Plummer half-mass radius is a / sqrt(2^(2/3) - 1) with a = 3 pi / 16
    in Henon units; the kinetic energy is 1/4."""
    x, v = workloads.plummer(65536, 3)
    r = np.linalg.norm(x, axis=1)
    rh = PLUMMER_LENGTH / np.sqrt(2 ** (2 / 3) - 1)
    assert np.median(r) == pytest.approx(rh, rel=0.02)
    assert 0.5 * np.mean(np.sum(v * v, axis=1)) == pytest.approx(0.25, rel=0.02)


def test_salpeter_bounds_and_slope():
    m = workloads.salpeter_masses(200000, 5)
    assert m.sum() == pytest.approx(1.0, rel=1e-12)
    ratio = m / m.min()
    assert ratio.max() <= 1000.0 * (1 + 1e-9)
    # log-histogram slope of dN/dlogm is slope + 1 = -1.35
    raw = m / m.sum() * 1.0
    lm = np.log10(raw / raw.min() * 0.1)
    hist, edges = np.histogram(lm, bins=12, range=(-1, 2))
    centres = 0.5 * (edges[1:] + edges[:-1])
    ok = hist > 50
    slope = np.polyfit(centres[ok], np.log10(hist[ok]), 1)[0]
    assert slope == pytest.approx(-1.35, abs=0.08)


def test_binaries_have_drawn_elements():
    rng = np.random.default_rng(9)
    nb = 500
    m1 = m2 = 1.0 / 4096
    cx = rng.normal(size=(nb, 3)); cv = rng.normal(size=(nb, 3))
    x, v, a, e = workloads.hard_binaries(cx, cv, m1, m2, 11)
    assert np.all((a >= 1e-5) & (a <= 1e-3)) and np.all((e >= 0) & (e < 1))
    r = x[1::2] - x[0::2]
    w = v[1::2] - v[0::2]
    mu = m1 + m2
    rn = np.linalg.norm(r, axis=1)
    # vis-viva: 1/a = 2/r - w^2/mu ; eccentricity vector from the relative orbit
    a_rec = 1.0 / (2.0 / rn - np.sum(w * w, axis=1) / mu)
    evec = (np.sum(w * w, axis=1) / mu - 1 / rn)[:, None] * r - (np.sum(r * w, axis=1) / mu)[:, None] * w
    np.testing.assert_allclose(a_rec, a, rtol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(evec, axis=1), e, atol=1e-9)
    # centre of mass of each pair sits on its centre
    np.testing.assert_allclose(0.5 * (x[0::2] + x[1::2]), cx, atol=1e-15)


def test_config_c5_layout():
    jm = workloads.config_c5(n=2 ** 12)
    assert jm.n == 2 ** 12
    nb = jm.meta["n_binaries"]
    assert nb == round(0.025 * 2 ** 12)
    assert jm.meta["is_binary"].sum() == 2 * nb
    assert np.allclose(jm.x.mean(axis=0), 1e4, atol=1.0)
    assert jm.meta["eps2"] == 0.0


def test_config_c3_small_and_active_sets():
    jm = workloads.config_c3(n=4096)
    assert jm.m.sum() == pytest.approx(1.0)
    assert jm.meta["ti"] == 2.0 ** -10 and jm.meta["eps2"] == 1e-8
    s = workloads.active_set(4096, 100, 3)
    assert s.size == 100 and np.all(np.diff(s) > 0)
    assert np.array_equal(s, workloads.active_set(4096, 100, 3))


def test_digest_is_stable():
    jm = workloads.config_c1()
    assert workloads.input_digest(jm.x, jm.v) == workloads.input_digest(jm.x.copy(), jm.v.copy())
