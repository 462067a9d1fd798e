"""Pins of the CPU bridge oracle (second-order Hamiltonian split of a
collisional subsystem c and a field subsystem g): the field across the split
adds up to the whole, kicks conserve momentum, the two-body split is the
textbook leapfrog and converges at second order, massless c leaves g a plain
leapfrog, and a cluster-in-galaxy system self-converges at second order in
the bridge step with a small energy error."""
import numpy as np

import oracle
from oracle import bridge as B
import synth


def _split(n=300, n_c=24, seed=11):
    p = synth.plummer(n, seed)
    r = np.linalg.norm(p.pos, axis=1)
    order = np.argsort(r, kind="stable")
    c, g = np.sort(order[:n_c]), np.sort(order[n_c:])
    return p, g, c


def test_cross_field_adds_up_to_the_whole():
    p, g, c = _split()
    eps2 = 1e-3
    a_full, j_full, p_full, _ = oracle.forces_f64(p.pos, p.vel, p.mass, eps2, c.astype(np.int32))
    a_cc, j_cc, p_cc, _ = oracle.forces_f64(p.pos[c], p.vel[c], p.mass[c], eps2)
    a_cg, j_cg, p_cg = B.cross_forces(p.pos[c], p.vel[c], p.pos[g], p.vel[g], p.mass[g], eps2)
    for whole, part1, part2 in ((a_full, a_cc, a_cg), (j_full, j_cc, j_cg), (p_full, p_cc, p_cg)):
        err = np.linalg.norm(part1 + part2 - whole) / np.linalg.norm(whole)
        assert err < 1e-14, err
    # the receiving particles exert nothing: moving them leaves the field of g unchanged
    a2 = B.cross_forces(p.pos[c] + 0.01, p.vel[c], p.pos[g], p.vel[g], p.mass[g], eps2)[0]
    a_shift = oracle.forces_f64(np.concatenate([p.pos[g], p.pos[c] + 0.01]), np.concatenate([p.vel[g], p.vel[c]]),
                                np.concatenate([p.mass[g], np.zeros(c.size)]), eps2,
                                np.arange(g.size, g.size + c.size, dtype=np.int32))[0]
    np.testing.assert_array_equal(a2, a_shift)


def test_kicks_conserve_total_momentum_and_keep_positions():
    p, g, c = _split()
    st = B.initialise(p.pos[g], p.vel[g], p.mass[g], p.pos[c], p.vel[c], p.mass[c], 1e-3, 1e-4, 1e-3, 1.0 / 64)
    mom = lambda: (st.mg[:, None] * st.vg).sum(0) + (st.cluster.m[:, None] * st.cluster.v).sum(0)
    scale = (st.mg[:, None] * np.abs(st.vg)).sum() + (st.cluster.m[:, None] * np.abs(st.cluster.v)).sum()
    P0, xg0, xc0, vc0 = mom(), st.xg.copy(), st.cluster.x.copy(), st.cluster.v.copy()
    B.kick(st, 0.05)
    assert np.abs(mom() - P0).max() < 1e-15 * scale
    np.testing.assert_array_equal(st.xg, xg0)
    np.testing.assert_array_equal(st.cluster.x, xc0)
    assert np.abs(st.cluster.v - vc0).max() > 1e-6          # the kick did act


def _kepler_pair(e=0.5):
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


def test_two_body_split_is_the_textbook_leapfrog():
    # g = {body 0}, c = {body 1}: H_A is the whole interaction and both drifts
    # are free flights, so the split is the kick-drift-kick leapfrog.
    x, v, m = _kepler_pair()
    eps2, h = 1e-3, 2 * np.pi / 200
    st = B.initialise(x[:1], v[:1], m[:1], x[1:], v[1:], m[1:], 0.0, 0.0, eps2, h)
    X, V = x.copy(), v.copy()

    def acc(X):
        r = X[1] - X[0]
        f = r / (r @ r + eps2) ** 1.5
        return np.array([m[1] * f, -m[0] * f])

    for _ in range(60):
        V = V + 0.5 * h * acc(X)
        X = X + h * V
        V = V + 0.5 * h * acc(X)
        B.step(st)
    np.testing.assert_allclose(np.concatenate([st.xg, st.cluster.x]), X, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.concatenate([st.vg, st.cluster.v]), V, rtol=0, atol=1e-12)


def test_two_body_split_converges_at_second_order():
    errs = []
    t_end = 2 * np.pi * 1.3
    for n in (128, 256, 512, 1024):
        x, v, m = _kepler_pair()
        dt = 2 * np.pi / n
        st = B.initialise(x[:1], v[:1], m[:1], x[1:], v[1:], m[1:], 0.0, 0.0, 0.0, dt, max_level=4)
        steps = int(round(t_end / dt))
        for _ in range(steps):
            B.step(st)
        rel = st.cluster.x[0] - st.xg[0]
        errs.append(np.linalg.norm(rel - _kepler_rel(steps * dt)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 1.8) and np.all(slopes < 2.2), (errs, slopes)


def test_massless_cluster_leaves_the_galaxy_a_plain_leapfrog():
    p, g, c = _split(n=200, n_c=10, seed=5)
    eps2, dt, n_sub = 1e-3, 1.0 / 64, 2
    st = B.initialise(p.pos[g], p.vel[g], p.mass[g], p.pos[c], p.vel[c], np.zeros(c.size), eps2, eps2, eps2, dt,
                      n_sub=n_sub)
    X, V = p.pos[g].copy(), p.vel[g].copy()
    act = np.arange(g.size, dtype=np.int32)
    A = oracle.forces_f64(X, V, p.mass[g], eps2, act)[0]
    h = dt / n_sub
    for _ in range(5):
        for _ in range(n_sub):
            V = V + (0.5 * h) * A
            X = X + h * V
            A = oracle.forces_f64(X, V, p.mass[g], eps2, act)[0]
            V = V + (0.5 * h) * A
        B.step(st)
    np.testing.assert_array_equal(st.xg, X)
    np.testing.assert_array_equal(st.vg, V)


def test_cluster_in_galaxy_converges_at_second_order_in_the_bridge_step():
    # A galaxy with a heavy central particle; c is it and its innermost stars.
    # Self-convergence: the state at t = 1/8 moves by a quarter as much when
    # the bridge step halves (a first-order split would give a half).
    p, g, c = _split(n=240, n_c=16, seed=21)
    mass = p.mass.copy()
    mass[c[np.argmin(np.linalg.norm(p.pos[c], axis=1))]] = 0.02
    eps2 = 1e-3
    xs, drift = [], []
    for dt in (1.0 / 64, 1.0 / 128, 1.0 / 256):
        st = B.initialise(p.pos[g], p.vel[g], mass[g], p.pos[c], p.vel[c], mass[c], eps2, eps2, eps2, dt,
                          eta=0.001, max_level=20)
        E0 = B.energy(st)["E"]
        for _ in range(int(round(0.125 / dt))):
            B.step(st)
        xs.append(np.concatenate([st.xg, st.cluster.x]))
        drift.append(abs(B.energy(st)["E"] - E0) / abs(E0))
    d1, d2 = np.abs(xs[0] - xs[1]).max(), np.abs(xs[1] - xs[2]).max()
    assert 3.6 < d1 / d2 < 4.4, (d1, d2)
    assert max(drift) < 1e-4, drift


def test_tree_cross_field_at_theta_zero_is_the_direct_bridge():
    # cross = "tree": the field of g on c comes from g's tree code on [g | c]
    # with c massless.  At theta = 0 the tree opens every leaf, so the bridge
    # equals the direct-sum bridge to rounding, and c exerts nothing on g in
    # that evaluation (g's own forces are those of the tree over g alone).
    p, g, c = _split(n=260, n_c=20, seed=23)
    eps2, dt = 1e-3, 1.0 / 64
    args = (p.pos[g], p.vel[g], p.mass[g], p.pos[c], p.vel[c], p.mass[c], eps2, 1e-4, eps2, dt)
    a = B.initialise(*args, eta=0.01, max_level=20)
    b = B.initialise(*args, eta=0.01, max_level=20, field=B.tree_field(eps2, 0.0), cross="tree", theta=0.0)
    ag_tree = B.tree_field(eps2, 0.0)(p.pos[g], p.mass[g])
    assert np.abs(b.ag - ag_tree).max() <= 1e-13 * np.abs(ag_tree).max()
    for _ in range(3):
        B.step(a)
        B.step(b)
    np.testing.assert_array_equal(a.cluster.level, b.cluster.level)
    for x, y in ((a.xg, b.xg), (a.vg, b.vg), (a.cluster.x, b.cluster.x), (a.cluster.v, b.cluster.v)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_tree_cross_field_conserves_energy_and_needs_one_softening():
    import pytest
    p, g, c = _split(n=260, n_c=20, seed=24)
    eps2, dt = 1e-3, 1.0 / 64
    args = (p.pos[g], p.vel[g], p.mass[g], p.pos[c], p.vel[c], p.mass[c], eps2, 1e-4)
    with pytest.raises(ValueError):
        B.initialise(*args, 2 * eps2, dt, cross="tree")
    st = B.initialise(*args, eps2, dt, eta=0.01, max_level=20, field=B.tree_field(eps2, 0.5), cross="tree",
                      theta=0.5)
    E0 = B.energy(st)["E"]
    for _ in range(8):
        B.step(st)
    assert abs(B.energy(st)["E"] - E0) < 1e-4 * abs(E0)
