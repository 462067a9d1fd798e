"""Pins of the CPU tree-code oracle: the Peano-Hilbert keys (a bijection whose
consecutive indices are grid neighbours and whose prefixes are aligned
cubes), the tree (leaves partition the particles, cubes contain their
particles), the moments (definitions, parallel-axis consistency, the
far-field acceleration error falling as the fifth power of the distance), the opening
criterion (no accepted cell touches its group), theta = 0 reproducing the
direct sum, and the force error falling with theta."""
import numpy as np
import pytest

import oracle
from oracle import tree as TR
import synth


def _grid(bits):
    r = np.arange(2 ** bits)
    return np.array(np.meshgrid(r, r, r, indexing="ij")).reshape(3, -1).T


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_keys_are_a_bijection_along_unit_steps(bits):
    g = _grid(bits)
    k = TR.hilbert_keys(g, bits)
    assert sorted(k.tolist()) == list(range(8 ** bits))
    o = np.argsort(k)
    steps = np.abs(np.diff(g[o], axis=0))
    assert np.all(steps.sum(1) == 1)           # one unit step along one axis
    assert k[0] == 0                            # the curve starts at the origin


def test_hilbert_prefixes_are_aligned_cubes():
    bits = 4
    g = _grid(bits)
    k = TR.hilbert_keys(g, bits)
    for level in range(1, bits):
        side = 2 ** (bits - level)
        pre = k >> (3 * (bits - level))
        for p in np.unique(pre):
            pts = g[pre == p]
            lo = pts.min(0)
            assert len(pts) == side ** 3
            assert np.all(pts.max(0) - lo == side - 1) and np.all(lo % side == 0)


def test_tree_leaves_partition_and_cubes_contain():
    p = synth.plummer(3000, 2)
    t = TR.build(p.pos, p.mass, n_crit=16)
    covered = np.zeros(3000, dtype=int)
    for c in t.cells:
        x = t.pos[c.begin:c.end]
        assert np.all(x >= c.corner - 1e-12) and np.all(x <= c.corner + c.side + 1e-12)
        if c.leaf:
            covered[c.begin:c.end] += 1
            assert c.end - c.begin <= 16 or c.level == TR.LEAF_LEVEL
        else:
            kids = [t.cells[i] for i in c.children]
            assert kids[0].begin == c.begin and kids[-1].end == c.end
            assert all(a.end == b.begin for a, b in zip(kids, kids[1:]))
    assert np.all(covered == 1)
    assert sorted(t.order.tolist()) == list(range(3000))


def test_moments_definitions_and_parallel_axis():
    p = synth.plummer(2000, 3)
    t = TR.build(p.pos, p.mass, n_crit=16)
    for c in t.cells[:50]:
        if c.leaf:
            continue
        kids = [t.cells[i] for i in c.children]
        M = sum(k.M for k in kids)
        X = sum(k.M * k.X for k in kids) / M
        Q = sum(k.Q + k.M * (3 * np.outer(k.X - X, k.X - X) - np.dot(k.X - X, k.X - X) * np.eye(3)) for k in kids)
        assert M == pytest.approx(c.M, rel=1e-14)
        np.testing.assert_allclose(X, c.X, rtol=0, atol=1e-14)
        np.testing.assert_allclose(Q, c.Q, rtol=0, atol=1e-13 * np.abs(c.Q).max())
        assert abs(np.trace(c.Q)) <= 1e-13 * np.abs(c.Q).max()
        np.testing.assert_allclose(c.Q, c.Q.T, rtol=0, atol=0)


def test_multipole_far_field_error_falls_as_the_fifth_power():
    # A lumpy cluster seen from distances R and 2R: the error of the
    # quadrupole-truncated acceleration is the octupole term's gradient,
    # ~ R^-5 (ratio 32); a wrong or missing quadrupole term leaves ~ R^-4.
    rng = np.random.default_rng(4)
    x = rng.standard_normal((200, 3)) * np.array([1.0, 0.5, 0.3])
    m = rng.uniform(0.5, 1.5, 200)
    t = TR.build(x, m, n_crit=1000)                     # the root is one leaf with all the mass
    c = t.cells[0]
    errs = []
    direction = np.array([0.6, -0.48, 0.64])
    for R in (40.0, 80.0):
        xi = c.X + R * direction
        a_mp = TR.cell_field(c.M, c.X, c.Q, xi[None, :], 0.0)[0][0]
        r = x - xi
        a_dir = (m[:, None] * r / ((r * r).sum(1) ** 1.5)[:, None]).sum(0)
        errs.append(np.linalg.norm(a_mp - a_dir))
        mono = np.linalg.norm(c.M * (c.X - xi) / np.linalg.norm(c.X - xi) ** 3 - a_dir)
        assert errs[-1] < 0.05 * mono                   # the quadrupole term does its job
    assert 24 < errs[0] / errs[1] < 36, errs


def test_opening_criterion_never_accepts_a_cell_touching_its_group():
    p = synth.plummer(4000, 5)
    t = TR.build(p.pos, p.mass, n_crit=16)
    for g in TR.groups(t, t.side / 16)[::7]:
        ci, li = TR.walk(t, g, 0.7)
        b, e = g
        glo, ghi = t.pos[b:e].min(0), t.pos[b:e].max(0)
        for k in ci:
            c = t.cells[k]
            gap = np.maximum(np.maximum(c.corner - ghi, glo - (c.corner + c.side)), 0)
            assert np.linalg.norm(gap) > c.side / 0.7 * (1 - 1e-12)
        # accepted cells and opened leaves cover every particle exactly once
        cover = np.zeros(4000, dtype=int)
        for k in ci + li:
            cover[t.cells[k].begin:t.cells[k].end] += 1
        assert np.all(cover == 1)


def test_groups_are_contiguous_and_small():
    p = synth.plummer(5000, 6)
    t = TR.build(p.pos, p.mass)
    gs = TR.groups(t, t.side / 16)
    assert gs[0][0] == 0 and gs[-1][1] == 5000
    assert all(a[1] == b[0] for a, b in zip(gs, gs[1:]))
    for b, e in gs:
        assert 1 <= e - b <= 64
        ext = (t.pos[b:e].max(0) - t.pos[b:e].min(0)).max()
        assert ext <= t.side / 16 or e - b == 1


def test_theta_zero_is_the_direct_sum():
    p = synth.plummer(1500, 7)
    eps2 = 1e-3
    acc, pot, _ = TR.forces(p.pos, p.mass, eps2, theta=0.0)
    a_ref, _, p_ref, _ = oracle.forces_f64(p.pos, p.vel, p.mass, eps2)
    assert np.linalg.norm(acc - a_ref) <= 1e-13 * np.linalg.norm(a_ref)
    assert np.linalg.norm(pot - p_ref) <= 1e-13 * np.linalg.norm(p_ref)


def test_force_error_falls_with_theta():
    p = synth.plummer(4000, 8)
    eps2 = 1e-4
    a_ref, _, p_ref, _ = oracle.forces_f64(p.pos, p.vel, p.mass, eps2)
    errs, work = [], []
    for theta in (0.8, 0.5, 0.3):
        acc, pot, st = TR.forces(p.pos, p.mass, eps2, theta)
        rel = np.linalg.norm(acc - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
        errs.append(np.sqrt(np.mean(rel ** 2)))
        work.append(sum(c + d for c, _, d in st))
    assert errs[0] > errs[1] > errs[2] and errs[0] > 5 * errs[2], errs
    assert errs[0] < 2e-3 and errs[2] < 1e-4, errs
    assert work[0] < work[1] < work[2] < 4000 * 4000
