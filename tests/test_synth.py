"""Pins of the seeded input generators against the distributions they sample.

Every expected value here comes from the model's own closed forms (cumulative
mass, the Plummer speed distribution, the energy integrals of a spherical
mass distribution) evaluated by quadrature, never from the generator's code;
statistical checks use five standard errors of the sample at hand.
"""
import numpy as np
import pytest
from scipy import integrate, optimize, special

import oracle
import synth

HENON_R = 3.0 * np.pi / 16.0          # Plummer scale length in Henon units
R_CUT = synth.PLUMMER_R_CUT            # radii beyond this (scale units) are redrawn


def _plummer_M(rho):
    """Mass inside rho (scale units) of a unit-mass Plummer sphere."""
    return rho ** 3 / (1.0 + rho * rho) ** 1.5


F_CUT = _plummer_M(R_CUT)


def _binomial_ok(frac, p, n, k=5.0):
    return abs(frac - p) <= k * np.sqrt(p * (1 - p) / n) + 1.0 / n


def test_generators_are_deterministic_per_seed():
    a, b, c = synth.plummer(1000, 7), synth.plummer(1000, 7), synth.plummer(1000, 8)
    for f in ("pos", "vel", "mass"):
        assert getattr(a, f).tobytes() == getattr(b, f).tobytes()
    assert not np.array_equal(a.pos, c.pos)
    x, y = synth.cluster_batch(4, 8), synth.cluster_batch(4, 8)
    for f in ("offsets", "eps2", "pos", "vel", "mass"):
        assert getattr(x, f).tobytes() == getattr(y, f).tobytes()
    assert not np.array_equal(synth.cluster_batch(5, 8).sizes, x.sizes)
    m1 = synth.hernquist_merger(5, n_gal=3, n_star=2048)
    m2 = synth.hernquist_merger(5, n_gal=3, n_star=2048)
    for f in ("pos", "vel", "mass", "active"):
        assert getattr(m1, f).tobytes() == getattr(m2, f).tobytes()


@pytest.mark.parametrize("seed", [3, 11])
def test_plummer_radii_follow_the_truncated_cumulative_mass(seed):
    # Fraction of bodies within r (Henon units) against M(r/(3pi/16)) / M(10).
    n = 16384
    p = synth.plummer(n, seed)
    assert p.mass.sum() == pytest.approx(1.0, rel=1e-14)
    assert np.abs((p.mass[:, None] * p.pos).sum(0)).max() < 1e-15
    assert np.abs((p.mass[:, None] * p.vel).sum(0)).max() < 1e-15
    r = np.linalg.norm(p.pos, axis=1)
    for rr in (0.1, 0.3, 0.6, 1.0, 2.0, 4.0):
        expect = _plummer_M(rr / HENON_R) / F_CUT
        assert _binomial_ok(np.mean(r < rr), expect, n), (rr, np.mean(r < rr), expect)
    # half-mass radius of the truncated model (0.769 without the cut)
    rho_h = optimize.brentq(lambda x: _plummer_M(x) / F_CUT - 0.5, 0.1, 10.0)
    r_half = rho_h * HENON_R
    assert (2.0 ** (2.0 / 3.0) - 1.0) ** -0.5 * HENON_R == pytest.approx(0.769, abs=5e-4)
    # median's standard error: sqrt(1/4n) / (dF/dr at the median)
    dens = 3.0 * rho_h ** 2 / (1 + rho_h ** 2) ** 2.5 / F_CUT / HENON_R
    assert abs(np.median(r) - r_half) < 5.0 * 0.5 / np.sqrt(n) / dens, (np.median(r), r_half)
    assert r.max() <= R_CUT * HENON_R * (1 + 1e-12) + 0.05


@pytest.mark.parametrize("seed", [3, 11])
def test_plummer_energies_and_virial_ratio(seed):
    # Speeds: q has density ~ q^2 (1-q^2)^{7/2}, so E[q^2] = B(5/2,9/2)/B(3/2,9/2)
    # = 1/4 and E[v^2 | rho] = 2 E[q^2] (1+rho^2)^{-1/2} in scale units.  With
    # the Henon scaling K = (16/3pi)/4 * E[(1+rho^2)^{-1/2}] over the truncated
    # radii; W = -int M dM / r (spherical mass) for the truncated, renormalised
    # mass.  Without the cut these are 1/4 and -1/2.
    n = 16384
    p = synth.plummer(n, seed)
    dM = lambda x: 3.0 * x * x / (1 + x * x) ** 2.5
    Eq2 = special.beta(2.5, 4.5) / special.beta(1.5, 4.5)
    assert Eq2 == pytest.approx(0.25, rel=1e-12)
    assert integrate.quad(lambda q: q ** 4 * (1 - q * q) ** 3.5, 0, 1)[0] == \
        pytest.approx(0.5 * special.beta(2.5, 4.5), rel=1e-8)
    K_exp = 0.5 * (16.0 / (3 * np.pi)) * 2 * Eq2 * \
        integrate.quad(lambda x: (1 + x * x) ** -0.5 * dM(x), 0, R_CUT)[0] / F_CUT
    W_exp = -(16.0 / (3 * np.pi)) * integrate.quad(lambda x: _plummer_M(x) * dM(x) / x, 0, R_CUT)[0] / F_CUT ** 2
    assert (16.0 / (3 * np.pi)) * integrate.quad(lambda x: _plummer_M(x) * dM(x) / x, 0, np.inf)[0] == \
        pytest.approx(0.5, rel=1e-10)
    ke = 0.5 * (p.vel * p.vel).sum(1)                       # m = 1/n: K = mean(ke)
    K = ke.mean()
    assert abs(K - K_exp) < 5.0 * ke.std() / np.sqrt(n), (K, K_exp)
    W = oracle.pair_potential_energy(p.pos, p.mass, 0.0)
    # U-statistic: sd(W) ~ sd(phi(x)) / sqrt(n); the sum over pairs lacks the
    # n self terms, a factor (n-1)/n
    pot = oracle.forces_ld(p.pos, p.vel, p.mass, 0.0)["pot"]
    assert abs(W - W_exp * (n - 1) / n) < 5.0 * pot.std() / np.sqrt(n), (W, W_exp)
    Q = K / abs(W)
    assert abs(Q - 0.5) < 3.0 / np.sqrt(n), Q
    assert abs(K + W + 0.25) < 3.0 / np.sqrt(n), K + W


def _hernquist_F(r):
    """Mass fraction inside r of a Hernquist sphere (a = 1) cut at r = 10."""
    return (r / (r + 1.0)) ** 2 / (10.0 / 11.0) ** 2


def test_hernquist_galaxies_cumulative_mass_and_dispersion():
    n_star, n_gal = 1 << 15, 3
    m = synth.hernquist_merger(21, n_gal=n_gal, n_star=n_star)
    assert m.pos.shape == (n_gal * (n_star + 1), 3)
    assert m.eps2 == pytest.approx((0.05 * n_star ** (-1.0 / 3.0)) ** 2, rel=1e-14)
    v_in = np.sqrt(2.0 * n_gal / 20.0)
    for g in range(n_gal):
        base = g * (n_star + 1)
        bh = base + n_star
        assert m.bh_index[g] == bh
        c = m.pos[bh]
        assert np.linalg.norm(c) == pytest.approx(20.0, rel=1e-14)
        assert m.vel[bh] == pytest.approx(-v_in * c / 20.0, rel=1e-13, abs=1e-15)
        assert m.mass[bh] == pytest.approx(1e-3, rel=1e-14)
        assert m.mass[base:bh].sum() + m.mass[bh] == pytest.approx(1.0, rel=1e-13)
        x = m.pos[base:bh] - c
        v = m.vel[base:bh] - m.vel[bh]
        assert np.abs(x.mean(0)).max() < 1e-12 and np.abs(v.mean(0)).max() < 1e-13
        r = np.linalg.norm(x, axis=1)
        for rr in (0.05, 0.2, 0.5, 1.0, 3.0, 8.0):
            assert _binomial_ok(np.mean(r < rr), _hernquist_F(rr), n_star), (g, rr)
        assert r.max() < 10.0 + 0.05                        # cut at 10 before the centring shift
        # |v|^2 / v_c(r)^2 is chi-square with 3 dof over 3: mean 1, variance 2/3
        vc2 = r / (1.0 + r) ** 2
        ratio = (v * v).sum(1) / vc2
        assert abs(ratio.mean() - 1.0) < 5.0 * np.sqrt(2.0 / 3.0 / n_star), ratio.mean()


def test_merger_i_set_size_and_membership():
    # Full-size direct part: 11 galaxies of 2^17 stars.  Expected stars within
    # 0.05 of each point mass: n_star F(0.05) = 2^17 (0.05/1.05)^2 / (10/11)^2 ~ 360.
    m = synth.hernquist_merger()
    n_star, n_gal = 1 << 17, 11
    assert m.pos.shape[0] == 1441803
    expect = n_star * _hernquist_F(0.05)
    assert expect == pytest.approx(359.6, abs=0.1)
    act = m.active
    assert np.all(np.diff(act) > 0) and set(m.bh_index.tolist()) <= set(act.tolist())
    d = np.stack([np.linalg.norm(m.pos - m.pos[b], axis=1) for b in m.bh_index])   # (11, N)
    near = (d < 0.05).any(0)
    assert np.array_equal(np.nonzero(near)[0], act)
    for g in range(n_gal):
        cnt = int((d[g] < 0.05).sum()) - 1                  # the point mass itself
        assert abs(cnt - expect) < 5.0 * np.sqrt(expect), (g, cnt)
    total = act.size - n_gal
    assert abs(total - n_gal * expect) < 5.0 * np.sqrt(n_gal * expect), total


def test_cluster_batch_sizes_softening_and_clusters():
    b = synth.cluster_batch()
    assert b.sizes.size == 128 and b.offsets[0] == 0
    assert np.array_equal(np.diff(b.offsets), b.sizes)
    assert b.sizes.min() >= 128 and b.sizes.max() <= 16384
    assert b.eps2 == pytest.approx((0.05 * b.sizes.astype(float) ** (-1.0 / 3.0)) ** 2, rel=1e-14)
    # log-uniform sizes: u = log(N/128)/log(128) against U(0,1), Kolmogorov-Smirnov at 1%
    u = np.sort(np.log(b.sizes / 128.0) / np.log(128.0))
    k = np.arange(1, u.size + 1) / u.size
    D = max(np.max(k - u), np.max(u - (k - 1.0 / u.size)))
    assert D < 1.63 / np.sqrt(u.size), D
    for c in range(b.sizes.size):
        sl = slice(b.offsets[c], b.offsets[c + 1])
        assert b.mass[sl].sum() == pytest.approx(1.0, rel=1e-13)
        assert np.abs((b.mass[sl, None] * b.pos[sl]).sum(0)).max() < 1e-14
        assert np.abs((b.mass[sl, None] * b.vel[sl]).sum(0)).max() < 1e-14
