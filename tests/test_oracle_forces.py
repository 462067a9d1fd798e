"""Pins of the CPU force oracle against closed forms, invariants and
finite differences (none of them re-types the oracle's own sum)."""
import numpy as np
import pytest

import oracle
import synth


def _both(pos, vel, m, eps2, active=None):
    a, j, p, sk = oracle.forces_f64(pos, vel, m, eps2, active)
    r = oracle.forces_ld(pos, vel, m, eps2, active)
    return (a, j, p, sk), r


@pytest.mark.parametrize("eps2", [0.0, 0.3])
def test_two_body_closed_form_static(eps2):
    # Particle 1 at the origin, particle 2 on the x axis at distance d: the
    # field of a point mass, |a| = m d / (d^2+eps^2)^{3/2}, phi = -m/sqrt(d^2+eps^2).
    d, m1, m2 = 1.7, 0.25, 0.75
    pos = np.array([[0, 0, 0], [d, 0, 0]], float)
    vel = np.zeros((2, 3))
    m = np.array([m1, m2])
    for (a, j, p, _), r in [_both(pos, vel, m, eps2)]:
        for acc, pot in [(a, p), (r["acc"], r["pot"])]:
            s32 = (d * d + eps2) ** 1.5
            assert acc[0] == pytest.approx([m2 * d / s32, 0, 0], rel=1e-15, abs=1e-300)
            assert acc[1] == pytest.approx([-m1 * d / s32, 0, 0], rel=1e-15, abs=1e-300)
            assert pot[0] == pytest.approx(-m2 / np.sqrt(d * d + eps2), rel=1e-15)
            assert pot[1] == pytest.approx(-m1 / np.sqrt(d * d + eps2), rel=1e-15)


@pytest.mark.parametrize("eps2", [0.0, 0.05])
def test_two_body_jerk_radial_and_transverse(eps2):
    # Radial approach: a(t) = m x(t)/(x^2+eps2)^{3/2} along x, so
    # da/dt = m xdot (eps2 - 2 x^2)/(x^2+eps2)^{5/2}  (derivative of the closed form).
    x, u, m2 = 1.3, -0.4, 0.6
    pos = np.array([[0, 0, 0], [x, 0, 0]], float)
    vel = np.array([[0, 0, 0], [u, 0, 0]], float)
    m = np.array([0.0, m2])
    (a, j, p, _), r = _both(pos, vel, m, eps2, np.array([0], np.int32))
    expect = m2 * u * (eps2 - 2 * x * x) / (x * x + eps2) ** 2.5
    for jj in (j, r["jerk"]):
        assert jj[0] == pytest.approx([expect, 0, 0], rel=1e-14, abs=1e-300)
    # Transverse motion: r.u = 0, so the jerk is m u / s^{3/2} along u.
    vel = np.array([[0, 0, 0], [0, 0, 0.9]], float)
    (a, j, p, _), r = _both(pos, vel, m, eps2, np.array([0], np.int32))
    expect = m2 * 0.9 / (x * x + eps2) ** 1.5
    for jj in (j, r["jerk"]):
        assert jj[0] == pytest.approx([0, 0, expect], rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("eps2", [0.0, 0.01])
def test_cube_corners(eps2):
    # 8 equal masses on the corners of a cube of side L: every acceleration
    # points at the centre; per axis the pull of the corner at (0,0,0) is
    # m L [1/(L^2+e)^{3/2} + 2/(2L^2+e)^{3/2} + 1/(3L^2+e)^{3/2}] (one
    # edge neighbour, two face diagonals, one body diagonal across that axis).
    L, mm = 0.8, 0.125
    corners = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float) * L
    vel = np.zeros((8, 3)); m = np.full(8, mm)
    comp = mm * L * (1 / (L * L + eps2) ** 1.5 + 2 / (2 * L * L + eps2) ** 1.5 + 1 / (3 * L * L + eps2) ** 1.5)
    pot = -mm * (3 / np.sqrt(L * L + eps2) + 3 / np.sqrt(2 * L * L + eps2) + 1 / np.sqrt(3 * L * L + eps2))
    (a, j, p, _), r = _both(corners, vel, m, eps2)
    centre = np.full(3, L / 2)
    for acc, ph in [(a, p), (r["acc"], r["pot"])]:
        expect = np.sign(centre - corners) * comp
        np.testing.assert_allclose(acc, expect, rtol=1e-14)
        np.testing.assert_allclose(ph, pot, rtol=1e-14)


def test_newton_third_law():
    p = synth.plummer(512, 11)
    a, j, _, _ = oracle.forces_f64(p.pos, p.vel, p.mass, 1e-4)
    fa = (p.mass[:, None] * a).sum(0)
    fj = (p.mass[:, None] * j).sum(0)
    assert np.linalg.norm(fa) <= 1e-14 * (p.mass * np.linalg.norm(a, axis=1)).sum()
    assert np.linalg.norm(fj) <= 1e-14 * (p.mass * np.linalg.norm(j, axis=1)).sum()


def test_jerk_is_time_derivative_of_acceleration():
    # Move every particle on its straight line; central differences of the
    # acceleration (with one Richardson step) must reproduce the jerk.
    p = synth.plummer(64, 3)
    eps2 = 0.01
    act = np.arange(64, dtype=np.int32)

    def acc_at(h):
        return oracle.forces_ld(p.pos + h * p.vel, p.vel, p.mass, eps2, act)["acc"]

    h = 2.5e-4
    d1 = (acc_at(h) - acc_at(-h)) / (2 * h)
    d2 = (acc_at(h / 2) - acc_at(-h / 2)) / h
    fd = (4 * d2 - d1) / 3
    j = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)["jerk"]
    err = np.linalg.norm(fd - j, axis=1) / np.linalg.norm(j, axis=1)
    assert err.max() < 1e-8


def test_potential_gradient_is_acceleration():
    p = synth.plummer(48, 5)
    eps2 = 0.02
    h = 1e-4
    r0 = oracle.forces_ld(p.pos, p.vel, p.mass, eps2)
    for i in range(0, 48, 7):
        g = np.zeros(3)
        for ax in range(3):
            def phi(dx):
                q = p.pos.copy(); q[i, ax] += dx
                return oracle.forces_ld(q, p.vel, p.mass, eps2, np.array([i], np.int32))["pot"][0]
            # fourth-order central difference
            g[ax] = -(-phi(2 * h) + 8 * phi(h) - 8 * phi(-h) + phi(-2 * h)) / (12 * h)
        assert np.linalg.norm(g - r0["acc"][i]) <= 1e-7 * np.linalg.norm(r0["acc"][i])


def test_total_potential_energy_by_pairs():
    p = synth.plummer(300, 8)
    eps2 = 1e-3
    r = oracle.forces_ld(p.pos, p.vel, p.mass, eps2)
    W_half = 0.5 * (p.mass * r["pot"]).sum()
    W_pairs = oracle.pair_potential_energy(p.pos, p.mass, eps2)
    assert W_half == pytest.approx(W_pairs, rel=1e-14)


def test_scaling_homogeneity():
    # x -> lam x, v -> nu v, m -> mu m, eps -> lam eps:
    # a -> mu/lam^2 a, jdot -> mu nu/lam^3 jdot, phi -> mu/lam phi.
    p = synth.plummer(200, 9)
    eps2 = 4e-3
    lam, nu, mu = 2.5, 0.3, 7.0
    r0 = oracle.forces_ld(p.pos, p.vel, p.mass, eps2)
    r1 = oracle.forces_ld(lam * p.pos, nu * p.vel, mu * p.mass, lam * lam * eps2)
    np.testing.assert_allclose(r1["acc"], mu / lam ** 2 * r0["acc"], rtol=1e-12, atol=1e-12 * np.abs(r1["acc"]).max())
    np.testing.assert_allclose(r1["jerk"], mu * nu / lam ** 3 * r0["jerk"], rtol=1e-12, atol=1e-12 * np.abs(r1["jerk"]).max())
    np.testing.assert_allclose(r1["pot"], mu / lam * r0["pot"], rtol=1e-13)


def test_far_field_is_monopole():
    # A compact cluster seen from distance D pulls like its total mass at its
    # centre of mass, up to O((size/D)^2).
    p = synth.plummer(256, 10)
    pos = p.pos * 0.01
    D = 50.0
    probe = np.array([[D, 0.3 * D, -0.2 * D]])
    allp = np.vstack([pos, probe]); vel = np.zeros_like(allp)
    m = np.concatenate([p.mass, [0.0]])
    r = oracle.forces_ld(allp, vel, m, 0.0, np.array([256], np.int32))
    rv = -probe[0]
    expect = rv / np.linalg.norm(rv) ** 3
    assert np.linalg.norm(r["acc"][0] - expect) <= 1e-6 * np.linalg.norm(expect)
    assert r["pot"][0] == pytest.approx(-1 / np.linalg.norm(rv), rel=1e-6)


def test_permutation_equivariance_and_subset():
    p = synth.plummer(128, 12)
    perm = np.random.default_rng(0).permutation(128)
    act = np.array([5, 17, 17, 90], np.int32)   # duplicates allowed
    a0, j0, p0, _ = oracle.forces_f64(p.pos, p.vel, p.mass, 1e-3)
    inv = np.argsort(perm)
    a1, j1, p1, _ = oracle.forces_f64(p.pos[perm], p.vel[perm], p.mass[perm], 1e-3, inv[act])
    np.testing.assert_allclose(a1, a0[act], rtol=1e-12)
    np.testing.assert_allclose(j1, j0[act], rtol=1e-12)
    np.testing.assert_allclose(p1, p0[act], rtol=1e-13)


def test_self_excluded_by_index_and_coincident_pairs():
    pos = np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    vel = np.zeros((3, 3)); m = np.array([0.5, 0.25, 0.25])
    # eps2 > 0: the twin contributes -m/eps to phi and nothing to a.
    a, j, ph, sk = oracle.forces_f64(pos, vel, m, 0.25)
    assert sk == 0
    assert ph[0] == pytest.approx(-0.25 / 0.5 - 0.25 / np.sqrt(1.25), rel=1e-15)
    assert a[0, 0] == pytest.approx(0.25 / 1.25 ** 1.5, rel=1e-15)
    # eps2 = 0: the coincident pair is skipped (counted once per receiving row).
    a, j, ph, sk = oracle.forces_f64(pos, vel, m, 0.0)
    assert sk == 2
    assert ph[0] == pytest.approx(-0.25, rel=1e-15)
    r = oracle.forces_ld(pos, vel, m, 0.0)
    assert r["skipped"] == 2


def test_f64_agrees_with_extended_within_rounding():
    p = synth.plummer(1024, 1)
    eps2 = synth.plummer_eps2_c1()
    a, j, ph, _ = oracle.forces_f64(p.pos, p.vel, p.mass, eps2)
    r = oracle.forces_ld(p.pos, p.vel, p.mass, eps2)
    ea = np.linalg.norm(a - r["acc"], axis=1) / r["abs_acc"]
    ej = np.linalg.norm(j - r["jerk"], axis=1) / r["abs_jerk"]
    ep = np.abs(ph - r["pot"]) / r["abs_pot"]
    # N=1024 terms, a few roundings each: well under 1024 * 2^-53.
    assert ea.max() < 1e-13 and ej.max() < 1e-13 and ep.max() < 1e-13


def _mp_forces(pos, vel, m, eps2, dps=50):
    """The force sum of the method's definition (i/j sum of section
    'Optimizations for the GPU'; Plummer softening, G = 1), evaluated with
    50-digit mpmath numbers from the double inputs: an evaluation that
    shares nothing with the oracle's C code or its rounding."""
    import mpmath
    with mpmath.workdps(dps):
        mp = mpmath.mpf
        n = len(m)
        P = [[mp(float(c)) for c in row] for row in pos]
        V = [[mp(float(c)) for c in row] for row in vel]
        M = [mp(float(c)) for c in m]
        e2 = mp(float(eps2))
        out = []
        for i in range(n):
            a = [mp(0)] * 3
            jk = [mp(0)] * 3
            ph = mp(0)
            for j in range(n):
                if j == i:
                    continue
                r = [P[j][c] - P[i][c] for c in range(3)]
                u = [V[j][c] - V[i][c] for c in range(3)]
                s = r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + e2
                rs = mpmath.sqrt(s)
                ru = r[0] * u[0] + r[1] * u[1] + r[2] * u[2]
                for c in range(3):
                    a[c] += M[j] * r[c] / (s * rs)
                    jk[c] += M[j] * u[c] / (s * rs) - 3 * M[j] * ru * r[c] / (s * s * rs)
                ph -= M[j] / rs
            out.append(([float(x) for x in a], [float(x) for x in jk], float(ph)))
    acc = np.array([o[0] for o in out])
    jerk = np.array([o[1] for o in out])
    pot = np.array([o[2] for o in out])
    return acc, jerk, pot


@pytest.mark.parametrize("eps2", [0.0, 1e-2])
def test_mpmath_brute_force_small_sets(eps2):
    # Random sets of 2..8 particles with unequal masses: both oracle
    # evaluations agree with the 50-digit sum of the definition.  Per
    # particle, e = |got - exact| / |exact| and kappa = sum_j |term_j| / |exact|
    # (the condition of the sum).  Extended precision: e <= 1e-15 (kappa/8 times
    # that where the sum cancels).  Plain double: each term takes about ten
    # roundings and the sum n - 1 more, so e <= (n + 12) u max(1, kappa),
    # u = 2^-53 -- a dropped term, a wrong sign or index is off by O(1).
    rng = np.random.default_rng(2024)
    worst = 0.0
    for trial in range(24):
        n = 2 + trial % 7
        pos = rng.uniform(-1.0, 1.0, (n, 3))
        vel = rng.uniform(-0.5, 0.5, (n, 3))
        m = rng.uniform(0.1, 1.0, n)
        ea, ej, ep = _mp_forces(pos, vel, m, eps2)
        a, j, p, sk = oracle.forces_f64(pos, vel, m, eps2)
        r = oracle.forces_ld(pos, vel, m, eps2)
        assert sk == 0 and r["skipped"] == 0
        for k in range(n):
            for got_a, got_j, got_p, name in ((a, j, p, "f64"), (r["acc"], r["jerk"], r["pot"], "ld")):
                for got, ref, absum in ((got_a[k], ea[k], r["abs_acc"][k]), (got_j[k], ej[k], r["abs_jerk"][k]),
                                        (np.array([got_p[k]]), np.array([ep[k]]), r["abs_pot"][k])):
                    nrm = np.linalg.norm(ref)
                    err = np.linalg.norm(got - ref) / nrm
                    kappa = absum / nrm
                    if name == "ld":
                        bound = 1e-15 * max(1.0, kappa / 8.0)
                    else:
                        bound = (n + 12) * 2.0 ** -53 * max(1.0, kappa)
                    assert err <= bound, (trial, n, k, name, err, kappa)
                    worst = max(worst, err / bound)
    assert worst > 0.0   # the comparison really ran on rounded values
