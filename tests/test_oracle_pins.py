"""Pins for the CPU float64 oracle.

Each test checks the oracle against something other than its own formula:
closed-form configurations derived by hand, calculus identities evaluated by
finite differences of the oracle's own outputs (acc = -grad phi, jerk =
d acc / dt), exact symmetries (Newton's third law, rigid rotation,
homologous expansion), the Plummer model's known potential energy, a k-d
tree from scipy for the neighbour search, and exact rational arithmetic for
the predictor.  A dropped term, a sign error, a wrong power of r or a swapped
i/j operand fails at least one of them.
"""

from fractions import Fraction

import numpy as np
import pytest

import workloads


def _rot(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return q * np.sign(np.linalg.det(q))


# ------------------------------------------------------------- predictor

def test_predictor_exact_for_cubic_trajectory(oracle_mod):
    """Eq. (1)/(2), Sec. 2.2: a cubic trajectory x(t) = c0 + c1 t + c2 t^2 +
    c3 t^3 is reproduced exactly by its third-order Taylor expansion about
    t_k.  Dyadic coefficients make every value exactly representable, so
    the only admissible difference is float64 rounding (<= 4 ulp)."""
    rng = np.random.default_rng(11)
    n = 64
    c = rng.integers(-64, 64, size=(4, n, 3)) / 16.0
    tk = rng.integers(0, 16, n) / 64.0
    ti = 0.5
    # state at t_k from the trajectory's derivatives, in exact arithmetic
    x0 = np.empty((n, 3)); v0 = np.empty((n, 3)); a2 = np.empty((n, 3)); j6 = np.empty((n, 3))
    xe = np.empty((n, 3)); ve = np.empty((n, 3))
    for k in range(n):
        t = Fraction(tk[k]); T = Fraction(ti)
        for d in range(3):
            c0, c1, c2, c3 = (Fraction(c[p, k, d]) for p in range(4))
            x0[k, d] = float(c0 + c1 * t + c2 * t ** 2 + c3 * t ** 3)
            v0[k, d] = float(c1 + 2 * c2 * t + 3 * c3 * t ** 2)
            a2[k, d] = float((2 * c2 + 6 * c3 * t) / 2)
            j6[k, d] = float(6 * c3 / 6)
            xe[k, d] = float(c0 + c1 * T + c2 * T ** 2 + c3 * T ** 3)
            ve[k, d] = float(c1 + 2 * c2 * T + 3 * c3 * T ** 2)
    xp, vp = oracle_mod.predict(ti, tk, x0, v0, a2, j6)
    ulp = np.spacing(np.maximum(np.abs(xe), 1.0))
    assert np.all(np.abs(xp - xe) <= 4 * ulp)
    assert np.all(np.abs(vp - ve) <= 4 * np.spacing(np.maximum(np.abs(ve), 1.0)))


def test_predictor_identity_at_zero_step(oracle_mod):
    jm = workloads.random_cluster(100, seed=4)
    xp, vp = oracle_mod.predict(0.25, np.full(jm.n, 0.25), jm.x, jm.v, jm.a2, jm.j6)
    assert np.array_equal(xp, jm.x) and np.array_equal(vp, jm.v)


def test_predicted_velocity_is_time_derivative_of_position(oracle_mod):
    jm = workloads.random_cluster(50, seed=5)
    ti, h = 0.3, 1e-3
    f = [oracle_mod.predict(ti + s * h, jm.t, jm.x, jm.v, jm.a2, jm.j6)[0] for s in (-2, -1, 1, 2)]
    deriv = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
    _, vp = oracle_mod.predict(ti, jm.t, jm.x, jm.v, jm.a2, jm.j6)
    assert np.allclose(deriv, vp, rtol=1e-9, atol=1e-9)


# ------------------------------------------------------- closed forms

@pytest.mark.parametrize("eps", [0.0, 0.05, 0.3])
def test_two_body_closed_form(oracle_mod, eps):
    """One j-particle at distance d: |a| = m d / (d^2+eps^2)^{3/2} toward it,
    phi = -m / sqrt(d^2+eps^2).  Moving sideways with speed u gives
    jerk = m u / (d^2+eps^2)^{3/2} along the motion; moving apart with speed
    u gives jerk = m u (eps^2 - 2 d^2) / (d^2+eps^2)^{5/2} along the line of
    centres (d/dt of the radial magnitude)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        R = _rot(rng)
        d = rng.uniform(0.1, 3.0)
        m = rng.uniform(0.1, 2.0)
        u = rng.uniform(-1.0, 1.0)
        xi = rng.normal(size=3)
        s = d * d + eps * eps
        for kind in ("tangential", "radial"):
            vj = R @ (np.array([0.0, u, 0.0]) if kind == "tangential" else np.array([u, 0.0, 0.0]))
            xj = xi + R @ np.array([d, 0.0, 0.0])
            vi = rng.normal(size=3)
            res = oracle_mod.force(xj[None], (vj + vi)[None], [m], [1], xi[None], vi[None], [0], eps * eps)
            a_exp = R @ np.array([m * d / s ** 1.5, 0.0, 0.0])
            if kind == "tangential":
                j_exp = R @ np.array([0.0, m * u / s ** 1.5, 0.0])
            else:
                j_exp = R @ np.array([m * u * (eps * eps - 2 * d * d) / s ** 2.5, 0.0, 0.0])
            np.testing.assert_allclose(res["acc"][0], a_exp, rtol=1e-13, atol=1e-14 * np.linalg.norm(a_exp))
            np.testing.assert_allclose(res["jerk"][0], j_exp, rtol=1e-13, atol=1e-13 * (abs(m * u) / s ** 1.5))
            assert res["pot"][0] == pytest.approx(-m / np.sqrt(s), rel=1e-14)


def test_cube_corners_closed_form(oracle_mod):
    """Eight equal masses at the corners (+-L, +-L, +-L), eps = 0.  For the
    corner s*L (s in {-1,1}^3) the 3 edge, 3 face-diagonal and 1 body-
    diagonal neighbours give, per component,
        a_d = -s_d m / L^2 (1/4 + 1/(4 sqrt 2) + 1/(12 sqrt 3))
    and phi = -(m/L)(3/2 + 3/(2 sqrt 2) + 1/(2 sqrt 3))."""
    L, m = 0.75, 0.3
    s = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], dtype=float)
    x = s * L
    res = oracle_mod.force(x, np.zeros((8, 3)), np.full(8, m), np.arange(8), x, np.zeros((8, 3)), np.arange(8), 0.0)
    amag = m / L ** 2 * (0.25 + 1 / (4 * np.sqrt(2)) + 1 / (12 * np.sqrt(3)))
    np.testing.assert_allclose(res["acc"], -s * amag, rtol=1e-14)
    np.testing.assert_allclose(res["pot"], -(m / L) * (1.5 + 1.5 / np.sqrt(2) + 0.5 / np.sqrt(3)), rtol=1e-14)
    np.testing.assert_allclose(res["jerk"], 0.0, atol=0.0)


# -------------------------------------------------- calculus identities

def test_acceleration_is_minus_gradient_of_potential(oracle_mod):
    """a_i = -grad_{x_i} phi_i, by a 5-point central difference of the
    oracle's own potential with respect to the i-particle's position."""
    jm = workloads.random_cluster(40, seed=21)
    eps2 = 0.01
    ni = 8
    xi, vi, idx = jm.x[:ni].copy(), jm.v[:ni].copy(), jm.index[:ni]
    base = oracle_mod.force(jm.x, jm.v, jm.m, jm.index, xi, vi, idx, eps2)
    grad = np.zeros((ni, 3))
    h = 1e-4
    for d in range(3):
        vals = []
        for st in (-2, -1, 1, 2):
            xs = xi.copy(); xs[:, d] += st * h
            vals.append(oracle_mod.force(jm.x, jm.v, jm.m, jm.index, xs, vi, idx, eps2)["pot"])
        grad[:, d] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    scale = np.linalg.norm(base["acc"], axis=1, keepdims=True)
    assert np.all(np.abs(base["acc"] + grad) <= 1e-8 * scale)


@pytest.mark.parametrize("eps2", [0.0, 1e-3])
def test_jerk_is_time_derivative_of_acceleration(oracle_mod, eps2):
    """jerk_i = d a_i / dt when every particle moves on a straight line:
    the j-memory is predicted with zero a2 and j6 (x_k + v_k tau) and the
    i-particles are moved the same way; 5-point central difference in tau."""
    jm = workloads.random_cluster(60, seed=22)
    ni = 10
    zero = np.zeros_like(jm.x)
    t0 = np.zeros(jm.n)

    def acc_at(tau):
        xp, vp = oracle_mod.predict(tau, t0, jm.x, jm.v, zero, zero)
        return oracle_mod.force(xp, vp, jm.m, jm.index, xp[:ni], vp[:ni], jm.index[:ni], eps2)

    h = 1e-4
    f = [acc_at(s * h)["acc"] for s in (-2, -1, 1, 2)]
    deriv = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
    jerk = acc_at(0.0)["jerk"]
    scale = np.linalg.norm(jerk, axis=1, keepdims=True)
    assert np.all(np.abs(deriv - jerk) <= 1e-7 * scale)


def test_rigid_rotation_and_homologous_expansion(oracle_mod):
    """Velocities v = Omega x + H x (rigid rotation plus uniform expansion),
    eps = 0: every separation evolves as (1 + H t) R(t) r, so each
    acceleration evolves as R(t) a / (1 + H t)^2 and its derivative is
    jerk = Omega x a - 2 H a exactly.  The radial (r.w) term of the jerk is
    exercised by the expansion, the tangential one by the rotation."""
    rng = np.random.default_rng(3)
    x, _ = workloads.plummer(200, rng)
    m = workloads.salpeter_masses(200, rng)
    omega = np.array([0.3, -0.7, 0.5])
    for H in (0.0, 0.4, -0.9):
        v = np.cross(omega, x) + H * x
        res = oracle_mod.force(x, v, m, np.arange(200), x, v, np.arange(200), 0.0)
        expect = np.cross(omega, res["acc"]) - 2 * H * res["acc"]
        scale = np.abs(m[None, :] / np.maximum(1e-300, np.sum((x[None] - x[:, None]) ** 2, axis=2)) ** 1.0)
        bound = 1e-12 * (np.linalg.norm(omega) + abs(H)) * scale.sum(axis=1)
        assert np.all(np.linalg.norm(res["jerk"] - expect, axis=1) <= bound)


def test_rotation_with_softening(oracle_mod):
    """A pure rotation preserves every separation, so jerk = Omega x a for
    any softening."""
    rng = np.random.default_rng(8)
    x, _ = workloads.plummer(150, rng)
    m = np.full(150, 1 / 150)
    omega = np.array([-0.2, 0.9, 0.4])
    v = np.cross(omega, x)
    res = oracle_mod.force(x, v, m, np.arange(150), x, v, np.arange(150), 0.02)
    expect = np.cross(omega, res["acc"])
    assert np.allclose(res["jerk"], expect, rtol=0, atol=1e-12 * np.abs(res["acc"]).max())


# ------------------------------------------------------------ symmetry

@pytest.mark.parametrize("eps2", [0.0, 2.0 ** -12])
def test_newton_third_law(oracle_mod, eps2):
    """With all particles active, pairwise antisymmetry of the softened
    force gives sum m_i a_i = 0 and sum m_i jerk_i = 0."""
    jm = workloads.random_cluster(512, seed=9)
    xp, vp = oracle_mod.predict(jm.meta["ti"], jm.t, jm.x, jm.v, jm.a2, jm.j6)
    res = oracle_mod.force(xp, vp, jm.m, jm.index, xp, vp, jm.index, eps2)
    for key in ("acc", "jerk"):
        tot = (jm.m[:, None] * res[key]).sum(axis=0)
        assert np.all(np.abs(tot) <= 1e-13 * np.sum(jm.m * np.linalg.norm(res[key], axis=1)))


def test_plummer_potential_energy(oracle_mod):
    """An unsoftened Plummer sphere in Henon units has W = -1/2 and
    K = 1/4 (virial equilibrium); a finite sample scatters by O(N^-1/2)."""
    x, v = workloads.plummer(8192, 123)
    m = np.full(8192, 1 / 8192)
    res = oracle_mod.force(x, v, m, np.arange(8192), x, v, np.arange(8192), 0.0)
    kin, wpot, _ = oracle_mod.energies(m, v, res["pot"])
    assert wpot == pytest.approx(-0.5, rel=0.03)
    assert kin == pytest.approx(0.25, rel=0.04)
    assert -2 * kin / wpot == pytest.approx(1.0, rel=0.05)


# ------------------------------------------------ self / index semantics

def test_self_excluded_by_index_not_position(oracle_mod):
    """The i-particle's own j-slot is skipped by index.  A different particle
    at the very same position (eps > 0) still contributes, and the sum over
    the remaining slots equals the sum with the own slot deleted."""
    jm = workloads.random_cluster(64, seed=31)
    eps2 = 1e-2
    k = 17
    twin_x = np.concatenate([jm.x, jm.x[k:k + 1]])
    twin_v = np.concatenate([jm.v, jm.v[k:k + 1]])
    twin_m = np.concatenate([jm.m, [0.5]])
    twin_idx = np.concatenate([jm.index, [1000]])
    res = oracle_mod.force(twin_x, twin_v, twin_m, twin_idx, jm.x[k:k + 1], jm.v[k:k + 1], [k], eps2)
    keep = np.arange(65) != k
    ref = oracle_mod.force(twin_x[keep], twin_v[keep], twin_m[keep], twin_idx[keep],
                           jm.x[k:k + 1], jm.v[k:k + 1], [k], eps2)
    for key in ("acc", "jerk", "pot"):
        assert np.array_equal(res[key], ref[key])
    assert res["nn_index"][0] == 1000 and res["nn_r2"][0] == 0.0
    # the twin's contribution to phi is -0.5/eps
    no_twin = oracle_mod.force(jm.x[keep[:64]], jm.v[keep[:64]], jm.m[keep[:64]], jm.index[keep[:64]],
                               jm.x[k:k + 1], jm.v[k:k + 1], [k], eps2)
    assert res["pot"][0] - no_twin["pot"][0] == pytest.approx(-0.5 / np.sqrt(eps2), rel=1e-12)


def test_degenerate_pairs_counted(oracle_mod):
    x = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    res = oracle_mod.force(x, np.zeros((3, 3)), [1.0, 1.0, 1.0], [0, 1, 2], x[:1], np.zeros((1, 3)), [0], 0.0)
    assert res["n_degenerate"] == 1
    assert np.all(np.isfinite(res["acc"])) and res["acc"][0, 0] == pytest.approx(1.0)


def test_thread_count_does_not_change_bits(oracle_mod):
    jm = workloads.random_cluster(700, seed=41)
    n0 = oracle_mod.max_threads()
    try:
        oracle_mod.set_threads(1)
        a = oracle_mod.evaluate(jm, jm.meta["ti"], np.arange(jm.n), 1e-4, 0.05)
        oracle_mod.set_threads(max(2, n0))
        b = oracle_mod.evaluate(jm, jm.meta["ti"], np.arange(jm.n), 1e-4, 0.05)
    finally:
        oracle_mod.set_threads(n0)
    for key in ("acc", "jerk", "pot", "nn_index", "nn_r2", "nb_count", "nb_list"):
        assert np.array_equal(a[key], b[key])


# --------------------------------------------------- neighbour search

@pytest.mark.parametrize("case", ["c1", "cluster"])
def test_neighbours_against_kdtree(oracle_mod, case):
    """Nearest neighbour and neighbour lists against scipy's k-d tree."""
    from scipy.spatial import cKDTree
    if case == "c1":
        jm = workloads.config_c1()
        h2 = jm.meta["h2"]
    else:
        jm = workloads.random_cluster(3000, seed=51)
        h2 = 0.02
    res = oracle_mod.force(jm.x, jm.v, jm.m, jm.index, jm.x, jm.v, jm.index, 1e-4, h2)
    tree = cKDTree(jm.x)
    dist, nbr = tree.query(jm.x, k=2)
    assert np.array_equal(nbr[:, 0], np.arange(jm.n))  # self first, distance 0
    assert np.array_equal(res["nn_index"], nbr[:, 1])
    np.testing.assert_allclose(res["nn_r2"], dist[:, 1] ** 2, rtol=1e-12)
    balls = tree.query_ball_point(jm.x, np.sqrt(h2))
    for i in range(jm.n):
        ref = sorted(k for k in balls[i] if k != i)
        assert res["nb_count"][i] == len(ref)
        cnt = min(len(ref), 256)
        assert list(res["nb_list"][i, :cnt]) == ref[:cnt]
        assert np.all(res["nb_list"][i, cnt:] == -1)


def test_neighbour_list_overflow_keeps_smallest_indices(oracle_mod):
    """More neighbours than the cap: the true count is reported and the
    kept entries are the cap smallest particle indices, ascending."""
    rng = np.random.default_rng(61)
    n = 600
    x = rng.normal(size=(n, 3)) * 0.01
    idx = rng.permutation(np.arange(10, 10 + n)).astype(np.int32)
    res = oracle_mod.force(x, np.zeros((n, 3)), np.full(n, 1 / n), idx, x[:3], np.zeros((3, 3)), idx[:3], 0.0,
                           h2=1.0, nb_cap=256)
    for i in range(3):
        others = np.sort(idx[idx != idx[i]])
        assert res["nb_count"][i] == n - 1
        assert np.array_equal(res["nb_list"][i], others[:256])


def test_neighbour_radius_is_strict(oracle_mod):
    """A j-particle exactly on the sphere r2u == h2 (dyadic values, exact in
    float64) is not a neighbour; one just inside is."""
    x = np.array([[0.0, 0, 0], [0.5, 0, 0], [0, 0.5 - 2.0 ** -40, 0], [0, 0, 0.75]])
    res = oracle_mod.force(x, np.zeros((4, 3)), np.ones(4), [0, 1, 2, 3], x[:1], np.zeros((1, 3)), [0], 0.0,
                           h2=0.25, nb_cap=4)
    assert res["nb_count"][0] == 1 and list(res["nb_list"][0]) == [2, -1, -1, -1]


def test_nearest_neighbour_tie_takes_smaller_index(oracle_mod):
    x = np.array([[0.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0], [0, 2.0, 0]])
    res = oracle_mod.force(x, np.zeros((4, 3)), np.ones(4), [5, 9, 7, 1], x[:1], np.zeros((1, 3)), [5], 0.0)
    assert res["nn_index"][0] == 7 and res["nn_r2"][0] == 1.0
    res = oracle_mod.force(x[:1], np.zeros((1, 3)), [1.0], [5], x[:1], np.zeros((1, 3)), [5], 0.0)
    assert res["nn_index"][0] == -1 and res["nn_r2"][0] == np.inf


# -------------------------------------------------- high-precision check

def test_tiny_systems_against_50_digit_arithmetic(oracle_mod):
    """Brute force at 50 decimal digits (mpmath) for N <= 12: the float64
    oracle differs only by rounding."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(71)
    for n, eps2 in ((2, 0.0), (5, 0.01), (12, 1e-4)):
        x = rng.normal(size=(n, 3)); v = rng.normal(size=(n, 3)); m = rng.uniform(0.1, 1.0, n)
        res = oracle_mod.force(x, v, m, np.arange(n), x, v, np.arange(n), eps2)
        for i in range(n):
            A = [mp.mpf(0)] * 3; J = [mp.mpf(0)] * 3; P = mp.mpf(0)
            for k in range(n):
                if k == i:
                    continue
                r = [mp.mpf(x[k, d]) - mp.mpf(x[i, d]) for d in range(3)]
                w = [mp.mpf(v[k, d]) - mp.mpf(v[i, d]) for d in range(3)]
                s = sum(c * c for c in r) + mp.mpf(eps2)
                rw = sum(r[d] * w[d] for d in range(3))
                for d in range(3):
                    A[d] += mp.mpf(m[k]) * r[d] / s ** 1.5
                    J[d] += mp.mpf(m[k]) * (w[d] / s ** 1.5 - 3 * rw * r[d] / s ** 2.5)
                P -= mp.mpf(m[k]) / mp.sqrt(s)
            an = float(mp.sqrt(sum(c * c for c in A)))
            jn = float(mp.sqrt(sum(c * c for c in J)))
            assert np.all(np.abs(res["acc"][i] - np.array([float(c) for c in A])) <= 1e-13 * an)
            assert np.all(np.abs(res["jerk"][i] - np.array([float(c) for c in J])) <= 1e-12 * jn)
            assert abs(res["pot"][i] - float(P)) <= 1e-14 * abs(float(P))


def test_conditioning_sums(oracle_mod):
    """The magnitude sums bound the vector sums (triangle inequality) and
    equal them for a single pair."""
    jm = workloads.random_cluster(300, seed=81)
    res = oracle_mod.force(jm.x, jm.v, jm.m, jm.index, jm.x, jm.v, jm.index, 1e-3, conditioning=True)
    assert np.all(res["acc_abs"] >= np.linalg.norm(res["acc"], axis=1) * (1 - 1e-14))
    assert np.all(res["jerk_abs"] >= np.linalg.norm(res["jerk"], axis=1) * (1 - 1e-14))
    two = oracle_mod.force(jm.x[:2], jm.v[:2], jm.m[:2], [0, 1], jm.x[:1], jm.v[:1], [0], 1e-3, conditioning=True)
    assert two["acc_abs"][0] == pytest.approx(np.linalg.norm(two["acc"][0]), rel=1e-14)
    assert two["jerk_abs"][0] == pytest.approx(np.linalg.norm(two["jerk"][0]), rel=1e-14)
