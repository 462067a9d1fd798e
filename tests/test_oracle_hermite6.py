"""Pins of the CPU oracle of the 6th-order Hermite scheme: snap against a
finite difference of the (separately pinned) jerk, Newton's third law, the
quintic interpolation and corrector on polynomials, the predictor, hand
values of the step criteria, the Kepler convergence order and the
block-step invariants."""
import numpy as np
import pytest

import oracle
from oracle import hermite as H
from oracle import hermite6 as H6
import synth


def _random_set(n=6, seed=3):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    v = rng.standard_normal((n, 3)) * 0.5
    a = rng.standard_normal((n, 3)) * 0.3
    m = rng.uniform(0.5, 1.5, n)
    return x, v, a, m


def test_snap_oracle_acc_jerk_pot_are_the_plain_sums():
    p = synth.plummer(300, 4)
    rng = np.random.default_rng(0)
    acc_j = rng.standard_normal((300, 3))
    r6 = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, 1e-3)
    r4 = oracle.forces_ld(p.pos, p.vel, p.mass, 1e-3)
    for k in ("acc", "jerk", "pot"):
        assert np.linalg.norm(r6[k] - r4[k]) <= 1e-15 * np.linalg.norm(r4[k]), k


@pytest.mark.parametrize("eps2", [0.0, 0.05])
def test_snap_is_the_time_derivative_of_the_jerk(eps2):
    # Every particle moves with its own constant acceleration a_i over the
    # instant: X(t) = x + v t + a t^2/2, V(t) = v + a t.  The jerk of the
    # plain sums along that motion, differentiated by a fourth-order central
    # difference, must be the snap.
    x, v, a, m = _random_set()
    h = 1e-3

    def jerk(t):
        return oracle.forces_ld(x + v * t + a * t * t / 2, v + a * t, m, eps2)["jerk"]

    fd = (-jerk(2 * h) + 8 * jerk(h) - 8 * jerk(-h) + jerk(-2 * h)) / (12 * h)
    snap = oracle.snap_ld(x, v, a, m, eps2)["snap"]
    assert np.linalg.norm(snap - fd) <= 1e-9 * np.linalg.norm(snap)


def test_snap_obeys_newtons_third_law():
    p = synth.plummer(500, 8)
    rng = np.random.default_rng(1)
    acc_j = rng.standard_normal((500, 3))
    r = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, 1e-3)
    tot = (p.mass[:, None] * r["snap"]).sum(0)
    scale = (p.mass * np.linalg.norm(r["snap"], axis=1)).sum()
    assert np.abs(tot).max() <= 1e-14 * scale


def _quintic(rng, n=4):
    return rng.standard_normal((6, n, 3))       # A0..A5: a(t) = sum A_k t^k / k!


def _a_derivs(A, t):
    fact = [1, 1, 2, 6, 24, 120]
    a = sum(A[k] * t ** k / fact[k] for k in range(6))
    j = sum(A[k] * t ** (k - 1) / fact[k - 1] for k in range(1, 6))
    s = sum(A[k] * t ** (k - 2) / fact[k - 2] for k in range(2, 6))
    return a, j, s


def test_interpolation_recovers_a_quintic():
    rng = np.random.default_rng(5)
    A = _quintic(rng)
    dt = 0.3
    a0, j0, s0 = _a_derivs(A, 0.0)
    a1, j1, s1 = _a_derivs(A, dt)
    c0, p0, q0 = H6.interpolate(a0, j0, s0, a1, j1, s1, np.full(4, dt))
    np.testing.assert_allclose(c0, A[3], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(p0, A[4], rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(q0, A[5], rtol=1e-7, atol=1e-7)


def test_corrector_exact_for_quintic_acceleration():
    rng = np.random.default_rng(6)
    A = _quintic(rng)
    x0, v0 = rng.standard_normal((2, 4, 3))
    dt = 0.25
    fact = [1, 1, 2, 6, 24, 120, 720, 5040]
    v_exact = v0 + sum(A[k] * dt ** (k + 1) / fact[k + 1] for k in range(6))
    x_exact = x0 + v0 * dt + sum(A[k] * dt ** (k + 2) / fact[k + 2] for k in range(6))
    c_exact = A[3] + A[4] * dt + A[5] * dt * dt / 2
    p_exact = A[4] + A[5] * dt
    a0, j0, s0 = _a_derivs(A, 0.0)
    a1, j1, s1 = _a_derivs(A, dt)
    c0, p0, q0 = H6.interpolate(a0, j0, s0, a1, j1, s1, np.full(4, dt))
    x1, v1, c1, p1 = H6.correct(x0, v0, a0, j0, s0, c0, p0, q0, np.full(4, dt))
    np.testing.assert_allclose(x1, x_exact, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(v1, v_exact, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(c1, c_exact, rtol=1e-8, atol=1e-8)
    np.testing.assert_allclose(p1, p_exact, rtol=1e-7, atol=1e-7)


def test_predictor_exact_for_constant_crackle():
    rng = np.random.default_rng(7)
    x, v, a, j, s, c = rng.standard_normal((6, 5, 3))
    d = np.array([0.0, 0.1, 0.25, 0.5, 1.0])
    D = d[:, None]
    xp, vp, ap = H6.predict(x, v, a, j, s, c, d)
    np.testing.assert_allclose(xp, x + v * D + a * D ** 2 / 2 + j * D ** 3 / 6 + s * D ** 4 / 24 + c * D ** 5 / 120,
                               rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(vp, v + a * D + j * D ** 2 / 2 + s * D ** 3 / 6 + c * D ** 4 / 24, rtol=1e-14,
                               atol=1e-14)
    np.testing.assert_allclose(ap, a + j * D + s * D ** 2 / 2 + c * D ** 3 / 6, rtol=1e-14, atol=1e-14)


def test_step_criterion_hand_values():
    # sqrt(|a||s|) + |j| = sqrt(1*4) + 1 = 3; sqrt(|c||q|) + |p| = sqrt(1*9) + 5 = 8
    eta = 0.2
    one = lambda *v: np.array([v], dtype=np.float64)
    ds = H6.new_dt(one(1, 0, 0), one(0, 1, 0), one(4, 0, 0), one(1, 0, 0), one(0, 5, 0), one(0, 0, 9), eta, 1.0)
    assert ds[0] == pytest.approx(eta * (3.0 / 8.0) ** (1.0 / 3.0), rel=1e-15)
    z = np.zeros((1, 3))
    assert H6.new_dt(one(1, 0, 0), z, z, z, z, z, eta, 0.0625)[0] == 0.0625
    # start-up: |a|/|j| = 0.25, sqrt(|a|/|s|) = 1 -> 0.5 * 0.25 = 0.125 -> level 3
    lev, _ = H6.startup_level(one(2, 0, 0), one(0, 0, 8), one(0, 2, 0), 0.5, 1.0, 20)
    assert lev[0] == 3
    # start-up with no jerk uses the snap term alone: sqrt(2/8) = 0.5, 0.5 * 0.5 -> level 2
    lev, _ = H6.startup_level(one(2, 0, 0), z, one(0, 8, 0), 0.5, 1.0, 20)
    assert lev[0] == 2
    lev, _ = H6.startup_level(one(2, 0, 0), z, z, 0.5, 1.0, 20)
    assert lev[0] == 0


def _kepler_state(e=0.5):
    rp = 1 - e
    vp = np.sqrt((1 + e) / (1 - e))
    r = np.array([rp, 0, 0]); v = np.array([0, vp, 0])
    return np.array([-r / 2, r / 2]), np.array([-v / 2, v / 2]), np.array([0.5, 0.5])


def _kepler_rel(t, e=0.5):
    M = t % (2 * np.pi)
    E = M
    for _ in range(60):
        E -= (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return np.array([np.cos(E) - e, np.sqrt(1 - e * e) * np.sin(E), 0.0])


def test_kepler_sixth_order_convergence():
    errs = []
    t_end = 2 * np.pi * 1.3
    f = H6.oracle_forces6(0.0)
    for n in (96, 192, 384):
        dt = 2 * np.pi / n
        x, v, m = _kepler_state()
        act = np.arange(2, dtype=np.int32)
        a, j, _, _ = f(x, v, np.zeros_like(x), m, act)
        a, j, s, _ = f(x, v, a, m, act)
        c = np.zeros_like(a)
        steps = int(round(t_end / dt))
        for _ in range(steps):
            x, v, a, j, s, c = H6.shared_step(x, v, a, j, s, c, m, dt, f)
        errs.append(np.linalg.norm(x[1] - x[0] - _kepler_rel(steps * dt)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 5.5) and np.all(slopes < 6.6), (errs, slopes)


def test_block_step_invariants_and_energy():
    p = synth.plummer(128, 12)
    eps2, eta, dt_max, ML = 1e-3, 0.15, 1.0 / 16, 24
    f = H6.oracle_forces6(eps2)
    st = H6.initialise(p.pos, p.vel, p.mass, eps2, eta, 0.01, dt_max, ML, f)
    E0 = H.energy(st.x, st.v, st.m, oracle.forces_f64(st.x, st.v, st.m, eps2)[2])["E"]
    end = int(round(0.125 / st.tick))
    last, evals = -1, 0
    while int(st.t.min()) < end:
        t_next, act = H6.block_step(st, f)
        assert t_next > last
        last = t_next
        evals += act.size
        dt_ticks = np.left_shift(np.int64(1), (ML - st.level).astype(np.int64))
        assert np.all(st.t % dt_ticks == 0)
    assert np.all(st.t == end)
    assert evals == sum(st.n_active_hist)
    E1 = H.energy(st.x, st.v, st.m, oracle.forces_f64(st.x, st.v, st.m, eps2)[2])["E"]
    assert abs(E1 - E0) / abs(E0) < 1e-7
