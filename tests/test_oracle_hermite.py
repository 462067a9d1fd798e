"""Pins of the CPU Hermite oracle: exactness on polynomials, a hand-worked
time-step value, level rules, the Kepler convergence order, block-step
invariants and energy behaviour."""
import numpy as np
import pytest

import oracle
from oracle import hermite as H
import synth


def _cubic(t, c0, c1, c2, c3):
    return c0 + c1 * t + c2 * t * t / 2 + c3 * t ** 3 / 6


def test_predictor_exact_for_constant_jerk():
    rng = np.random.default_rng(1)
    x0, v0, a0, j0 = rng.standard_normal((4, 5, 3))
    d = 0.37
    xp, vp = H.predict(x0, v0, a0, j0, d)
    np.testing.assert_allclose(xp, _cubic(d, x0, v0, a0, j0), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(vp, v0 + a0 * d + j0 * d * d / 2, rtol=1e-14, atol=1e-14)
    # per-row offsets
    dd = np.array([0.1, 0.2, 0.0, 0.5, 1.0])
    xp, vp = H.predict(x0, v0, a0, j0, dd)
    np.testing.assert_allclose(xp, _cubic(dd[:, None], x0, v0, a0, j0), rtol=1e-14, atol=1e-14)


def test_corrector_exact_for_cubic_acceleration():
    # a(t) = A0 + A1 t + A2 t^2/2 + A3 t^3/6 integrates exactly to
    # x(t) = x0 + v0 t + A0 t^2/2 + A1 t^3/6 + A2 t^4/24 + A3 t^5/120.
    rng = np.random.default_rng(2)
    x0, v0, A0, A1, A2, A3 = rng.standard_normal((6, 4, 3))
    dt = 0.3
    a = lambda t: A0 + A1 * t + A2 * t * t / 2 + A3 * t ** 3 / 6
    jd = lambda t: A1 + A2 * t + A3 * t * t / 2
    x_exact = x0 + v0 * dt + A0 * dt ** 2 / 2 + A1 * dt ** 3 / 6 + A2 * dt ** 4 / 24 + A3 * dt ** 5 / 120
    v_exact = v0 + A0 * dt + A1 * dt ** 2 / 2 + A2 * dt ** 3 / 6 + A3 * dt ** 4 / 24
    xp, vp = H.predict(x0, v0, a(0), jd(0), dt)
    a2, a3 = H.interpolate(a(0), jd(0), a(dt), jd(dt), dt)
    np.testing.assert_allclose(a2, A2, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(a3, A3, rtol=1e-9, atol=1e-9)
    x1, v1 = H.correct(xp, vp, a2, a3, dt)
    np.testing.assert_allclose(x1, x_exact, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(v1, v_exact, rtol=1e-13, atol=1e-13)


def test_aarseth_hand_value():
    # a1=(1,0,0), jdot1=(0,1,0), a2 at the end (0,0,1), a3=(1,0,0):
    # num = 1*1 + 1 = 2, den = 1*1 + 1 = 2, so dt* = sqrt(eta).
    eta, dt = 0.01, 0.25
    a3 = np.array([[1.0, 0, 0]])
    a2 = np.array([[0.0, 0, 1]]) - a3 * dt
    ds = H.aarseth_dt(np.array([[1.0, 0, 0]]), np.array([[0.0, 1, 0]]), a2, a3, np.array([dt]), eta, 1.0)
    assert ds[0] == pytest.approx(np.sqrt(eta), rel=1e-15)
    # zero denominator (all derivatives zero) -> dt_max
    z = np.zeros((1, 3))
    assert H.aarseth_dt(np.array([[1.0, 0, 0]]), z, z, z, np.array([dt]), eta, 0.0625)[0] == 0.0625


def test_level_rules():
    dt_max, ML = 1.0, 10
    # halve until dt <= dt*: from level 1 (dt 0.5) with dt* = 0.1 -> level 4 (0.0625)
    lev, cl = H.new_level([1], [0.1], [1 << 9], dt_max, ML)
    assert lev[0] == 4 and not cl[0]
    # double once only when the new time is a multiple of 2 dt
    lev, _ = H.new_level([3], [10.0], [3 * (1 << 7)], dt_max, ML)  # t = 3 dt: not commensurate
    assert lev[0] == 3
    lev, _ = H.new_level([3], [10.0], [4 * (1 << 7)], dt_max, ML)  # t = 4 dt: commensurate
    assert lev[0] == 2
    lev, _ = H.new_level([0], [10.0], [1 << 10], dt_max, ML)       # never above dt_max
    assert lev[0] == 0
    # dt* in [dt, 2dt): keep
    lev, _ = H.new_level([2], [0.3], [1 << 8], dt_max, ML)
    assert lev[0] == 2
    # clamp at max_level
    lev, cl = H.new_level([9], [1e-9], [1 << 1], dt_max, ML)
    assert lev[0] == ML and cl[0]
    # startup: smallest k with dt_max 2^-k <= eta |a|/|j|
    lev, _ = H.startup_level(np.array([[2.0, 0, 0]]), np.array([[0, 0, 8.0]]), 0.5, 1.0, ML)
    assert lev[0] == 3   # target 0.125


def _kepler_state(e=0.5):
    # Relative orbit of two bodies of mass 1/2 each (G M = 1, a = 1, period
    # 2 pi), started at pericentre on the x axis.
    rp = 1 - e
    vp = np.sqrt((1 + e) / (1 - e))
    r = np.array([rp, 0, 0]); v = np.array([0, vp, 0])
    pos = np.array([-r / 2, r / 2]); vel = np.array([-v / 2, v / 2])
    return pos, vel, np.array([0.5, 0.5])


def _kepler_rel(t, e=0.5):
    # Kepler's equation M = E - e sin E, Newton-solved; pericentre on +x.
    M = t % (2 * np.pi)
    E = M if e < 0.8 else np.pi
    for _ in range(60):
        E -= (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return np.array([np.cos(E) - e, np.sqrt(1 - e * e) * np.sin(E), 0.0])


def _force_fn(eps2):
    def f(x, v, m, act):
        a, j, p, _ = oracle.forces_f64(x, v, m, eps2, act)
        return a, j, p
    return f


def test_kepler_fourth_order_convergence():
    errs = []
    t_end = 2 * np.pi * 1.3
    for n in (256, 512, 1024, 2048):
        dt = 2 * np.pi / n
        pos, vel, m = _kepler_state()
        f = _force_fn(0.0)
        a, j, _ = f(pos, vel, m, np.arange(2, dtype=np.int32))
        steps = int(round(t_end / dt))
        for _ in range(steps):
            pos, vel, a, j = H.shared_step(pos, vel, a, j, m, dt, f)
        rel = pos[1] - pos[0]
        errs.append(np.linalg.norm(rel - _kepler_rel(steps * dt)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 3.7) and np.all(slopes < 4.4), (errs, slopes)


def test_kepler_invariants_converge_at_fourth_order():
    # Energy, angular momentum and the direction of the Runge-Lenz vector of
    # the relative orbit (G M = 1) drift at the scheme's order: their errors
    # after 1.3 orbits fall about 16x per halving of the shared step (the
    # energy's from the second halving on, once the step resolves pericentre).
    def invariants(pos, vel):
        r, v = pos[1] - pos[0], vel[1] - vel[0]
        L = np.cross(r, v)
        A = np.cross(v, L) - r / np.linalg.norm(r)
        return 0.5 * (v @ v) - 1.0 / np.linalg.norm(r), L, np.arctan2(A[1], A[0])
    errs = {"E": [], "L": [], "peri": []}
    t_end = 2 * np.pi * 1.3
    for n in (256, 512, 1024, 2048):
        dt = 2 * np.pi / n
        pos, vel, m = _kepler_state()
        E0, L0, w0 = invariants(pos, vel)
        f = _force_fn(0.0)
        a, j, _ = f(pos, vel, m, np.arange(2, dtype=np.int32))
        for _ in range(int(round(t_end / dt))):
            pos, vel, a, j = H.shared_step(pos, vel, a, j, m, dt, f)
        E, L, w = invariants(pos, vel)
        errs["E"].append(abs(E - E0) / abs(E0))
        errs["L"].append(np.linalg.norm(L - L0) / np.linalg.norm(L0))
        errs["peri"].append(abs(w - w0))
    slope = {k: np.log2(np.array(v[:-1]) / np.array(v[1:])) for k, v in errs.items()}
    assert np.all(np.abs(slope["E"][1:] - 4) < 0.4), slope
    assert np.all(np.abs(slope["L"] - 4) < 0.4), slope
    assert np.all(np.abs(slope["peri"] - 4) < 0.4), slope


def _block_run(n, seed, eps2, eta, t_end=0.125, dt_max=1.0 / 16, max_level=24, check=None):
    p = synth.plummer(n, seed)
    f = _force_fn(eps2)
    st = H.initialise(p.pos, p.vel, p.mass, eps2, eta, dt_max, max_level, f)
    end_ticks = int(round(t_end / st.tick))
    last = -1
    while int(st.t.min()) < end_ticks:
        t_next, act = H.block_step(st, f)
        if check:
            check(st, t_next, act, last)
        last = t_next
    return p, st


def test_block_step_invariants():
    n = 256
    seen_sync = []

    def check(st, t_next, act, last):
        assert t_next > last                              # time moves forward
        dt_ticks = np.left_shift(np.int64(1), (st.max_level - st.level).astype(np.int64))
        assert np.all(st.t % dt_ticks == 0)               # t_i commensurate with dt_i
        assert np.all((st.level >= 0) & (st.level <= st.max_level))
        assert np.all(st.t <= t_next)
        assert np.all(st.t[act] == t_next)
        assert np.all(np.diff(act) > 0)                   # ascending, unique
        per_dtmax = 1 << st.max_level
        if t_next % per_dtmax == 0:                       # every multiple of dt_max syncs all
            assert act.size == n and np.all(st.t == t_next)
            seen_sync.append(t_next)

    p, st = _block_run(n, 21, 1e-3, 0.02, check=check)
    assert len(seen_sync) == 2
    assert sum(st.n_active_hist) + n == st.force_evals
    assert min(st.n_active_hist) >= 1 and st.steps > 10
    assert len(set(st.level.tolist())) > 1                # genuinely several levels


def _energy(p_or_x, v, m, eps2):
    r = oracle.forces_ld(p_or_x, v, m, eps2)
    return H.energy(p_or_x, v, m, r["pot"])


@pytest.mark.slow
def test_energy_drift_falls_with_eta():
    n, eps2 = 256, 1e-4
    drifts = []
    for eta in (0.04, 0.01):
        p, st = _block_run(n, 7, eps2, eta)
        e0 = _energy(p.pos, p.vel, p.mass, eps2)["E"]
        e1 = _energy(st.x, st.v, st.m, eps2)
        drifts.append(abs(e1["E"] - e0) / abs(e0))
        # momentum stays ~0 (exact in exact arithmetic for shared steps;
        # block steps break the symmetry only at O(dt^4))
        assert np.linalg.norm(e1["P"]) < 1e-6
    # dt scales as eta^{1/2} and the error as dt^4: a factor 4 in eta
    # should give ~16x; demand at least 4x.
    assert drifts[1] * 4 < drifts[0], drifts
    assert drifts[1] < 1e-5, drifts


def _circular_pair(m1=0.3, m2=0.9, d=1.5):
    """Two bodies on a circular orbit in the xy plane, centre of mass at rest
    at the origin (Kepler: relative speed sqrt(M/d)).  Returns x, v, m and the
    potentials phi_1 = -m2/d, phi_2 = -m1/d written out by hand."""
    M = m1 + m2
    v = np.sqrt(M / d)
    x = np.array([[-m2 / M * d, 0, 0], [m1 / M * d, 0, 0]])
    vv = np.array([[0, -m2 / M * v, 0], [0, m1 / M * v, 0]])
    m = np.array([m1, m2])
    pot = np.array([-m2 / d, -m1 / d])
    return x, vv, m, pot


def test_energy_circular_two_body_closed_form():
    # K = m1 m2 / (2d), W = -m1 m2 / d, P = 0 and L = m1 m2 sqrt(d/M) along +z
    # (the orbit turns counter-clockwise seen from +z).
    m1, m2, d = 0.3, 0.9, 1.5
    x, v, m, pot = _circular_pair(m1, m2, d)
    e = H.energy(x, v, m, pot)
    assert e["K"] == pytest.approx(m1 * m2 / (2 * d), rel=1e-15)
    assert e["W"] == pytest.approx(-m1 * m2 / d, rel=1e-15)
    assert e["E"] == pytest.approx(-m1 * m2 / (2 * d), rel=1e-15)
    assert np.abs(e["P"]).max() < 1e-16
    assert e["L"] == pytest.approx([0, 0, m1 * m2 * np.sqrt(d / (m1 + m2))], rel=1e-15, abs=1e-16)
    # W from the oracle's own potentials equals the hand value too
    r = oracle.forces_ld(x, v, m, 0.0)
    assert H.energy(x, v, m, r["pot"])["W"] == pytest.approx(-m1 * m2 / d, rel=1e-15)


def test_energy_rotated_and_boosted_pair():
    # Rotate by R, shift by X0 and boost by V: P = M V, L = R L0 + M X0 x V,
    # K = K0 + M |V|^2 / 2, W unchanged (fixes the order of the cross
    # product, the mass weighting of P and the halves in K and W).
    m1, m2, d = 0.3, 0.9, 1.5
    M = m1 + m2
    x, v, m, pot = _circular_pair(m1, m2, d)
    e0 = H.energy(x, v, m, pot)
    rng = np.random.default_rng(11)
    R, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(R) < 0:
        R[:, 0] = -R[:, 0]
    X0 = np.array([0.4, -1.1, 2.0])
    V = np.array([-0.3, 0.25, 0.7])
    e = H.energy(x @ R.T + X0, v @ R.T + V, m, pot)
    assert e["P"] == pytest.approx(M * V, rel=1e-14, abs=1e-15)
    assert e["L"] == pytest.approx(R @ e0["L"] + M * np.cross(X0, V), rel=1e-13, abs=1e-14)
    assert e["K"] == pytest.approx(e0["K"] + 0.5 * M * V @ V, rel=1e-14)
    assert e["W"] == pytest.approx(e0["W"], rel=1e-15)
