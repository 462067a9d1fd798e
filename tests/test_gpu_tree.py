"""GPU parity of the tree code against the CPU oracle, through the C ABI:
identical interaction sets (accepted cells and opened leaves per group) and
forces within rounding of the oracle's, theta = 0 reproducing the direct
sum, edge cases (one particle, coincident particles, two distant clusters,
unsoftened, leaves of one particle and of several hundred, a deep clustered
tree), repeatability, argument errors, and the mixed-precision force terms
within float rounding of the oracle."""
import numpy as np
import pytest

import oracle
from oracle import tree as TR
import synth

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def ctx():
    import paper_1409_5474_amd as nb
    c = nb.Context(0, "fp64")
    yield c
    c.close()


def _gpu(ctx, pos, mass, eps2, theta, n_crit=16, g_frac=1.0 / 16):
    import torch
    acc, pot, st = ctx.tree_forces(T(pos), T(mass), eps2, theta, n_crit, g_frac)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy(), st


def _oracle(pos, mass, eps2, theta, n_crit=16, g_frac=1.0 / 16):
    t = TR.build(pos, mass, n_crit)
    acc, pot, st = TR.forces(pos, mass, eps2, theta, n_crit, g_max=g_frac * t.side, tree=t)
    return acc, pot, st, t


U = 2.0 ** -53
COND = 64 * U


def _close(got, ref, tol, pos, mass, eps2):
    # normwise within tol, and per particle |d_i| <= tol |r_i| + COND A_i,
    # with A_i the magnitude sum over j of the direct-sum terms (from the
    # extended-precision oracle): a cell term's magnitude is within a few
    # times its members' sum, so A_i sets the scale of either side's
    # rounding, as in the direct-force gate
    a, p = got
    ra, rp = ref
    assert np.linalg.norm(a - ra) <= tol * np.linalg.norm(ra)
    assert np.linalg.norm(p - rp) <= tol * np.linalg.norm(rp)
    mag = oracle.forces_ld(pos, np.zeros_like(pos), mass, eps2)
    for d, r, A, name in ((np.linalg.norm(a - ra, axis=1), np.linalg.norm(ra, axis=1), mag["abs_acc"], "acc"),
                          (np.abs(p - rp), np.abs(rp), mag["abs_pot"], "pot")):
        worst = int(np.argmax(d - tol * r - COND * A))
        assert np.all(d <= tol * r + COND * A), (name, worst, d[worst], r[worst], A[worst])


@pytest.mark.parametrize("n,theta,n_crit,seed", [(3000, 0.5, 16, 1), (5000, 0.3, 8, 2), (4096, 0.8, 16, 3),
                                                 (2500, 0.6, 32, 4), (700, 0.5, 16, 5)])
def test_tree_matches_oracle(ctx, n, theta, n_crit, seed):
    p = synth.plummer(n, seed)
    eps2 = 1e-4
    acc, pot, st = _gpu(ctx, p.pos, p.mass, eps2, theta, n_crit)
    ra, rp, rst, t = _oracle(p.pos, p.mass, eps2, theta, n_crit)
    assert st["cells"] == len(t.cells)
    assert st["groups"] == len(rst)
    assert st["accepted"] == sum(c for c, _, _ in rst)
    assert st["opened_leaves"] == sum(l for _, l, _ in rst)
    assert st["depth"] == max(c.level for c in t.cells)
    _close((acc, pot), (ra, rp), 1e-12, p.pos, p.mass, eps2)


def test_theta_zero_is_the_direct_sum(ctx):
    import torch
    p = synth.plummer(2000, 7)
    eps2 = 1e-3
    acc, pot, st = _gpu(ctx, p.pos, p.mass, eps2, 0.0)
    assert st["accepted"] == 0
    a_ref, _, p_ref = ctx.forces(T(p.pos), T(p.vel), T(p.mass), T(np.arange(2000, dtype=np.int32)), eps2)
    torch.cuda.synchronize()
    _close((acc, pot), (a_ref.cpu().numpy(), p_ref.cpu().numpy()), 1e-13, p.pos, p.mass, eps2)


def test_one_particle_and_a_small_set(ctx):
    acc, pot, st = _gpu(ctx, np.array([[0.3, -0.2, 0.1]]), np.array([1.0]), 1e-3, 0.5)
    assert np.all(acc == 0) and np.all(pot == 0)
    assert st["cells"] == 1 and st["groups"] == 1
    p = synth.plummer(40, 8)
    acc, pot, st = _gpu(ctx, p.pos, p.mass, 1e-3, 0.5)
    ra, rp, _, _ = _oracle(p.pos, p.mass, 1e-3, 0.5)
    _close((acc, pot), (ra, rp), 1e-13, p.pos, p.mass, 1e-3)


def test_coincident_particles_and_two_distant_clusters(ctx):
    a = synth.plummer(1500, 9)
    b = synth.plummer(1500, 10)
    pos = np.concatenate([a.pos, b.pos * 0.5 + np.array([40.0, -25.0, 10.0])])
    mass = np.concatenate([a.mass, b.mass * 3.0])
    pos[17] = pos[1000]                      # two particles on one spot (softened)
    pos[2500] = pos[2501]
    acc, pot, st = _gpu(ctx, pos, mass, 1e-3, 0.6)
    ra, rp, rst, t = _oracle(pos, mass, 1e-3, 0.6)
    assert st["accepted"] == sum(c for c, _, _ in rst)
    assert st["depth"] == max(c.level for c in t.cells)
    _close((acc, pot), (ra, rp), 1e-12, pos, mass, 1e-3)


def test_unsoftened_distinct_positions(ctx):
    p = synth.plummer(3000, 11)
    acc, pot, st = _gpu(ctx, p.pos, p.mass, 0.0, 0.5)
    ra, rp, _, _ = _oracle(p.pos, p.mass, 0.0, 0.5)
    _close((acc, pot), (ra, rp), 1e-12, p.pos, p.mass, 0.0)


def test_groups_split_by_size(ctx):
    p = synth.plummer(3000, 12)
    _, _, st1 = _gpu(ctx, p.pos, p.mass, 1e-3, 0.5, g_frac=0.0)
    _, _, st2 = _gpu(ctx, p.pos, p.mass, 1e-3, 0.5, g_frac=1.0 / 64)
    t = TR.build(p.pos, p.mass)
    assert st1["groups"] == len(TR.groups(t, np.inf)) == (3000 + 63) // 64
    assert st2["groups"] == len(TR.groups(t, t.side / 64)) > st1["groups"]


def test_accuracy_against_direct_and_repeatability(ctx):
    import torch
    p = synth.plummer(65536, 13)
    eps2 = 2.0 ** -16
    acc1, pot1, st = _gpu(ctx, p.pos, p.mass, eps2, 0.5)
    acc2, pot2, _ = _gpu(ctx, p.pos, p.mass, eps2, 0.5)
    assert np.array_equal(acc1, acc2) and np.array_equal(pot1, pot2)
    a_ref, _, _ = ctx.forces(T(p.pos), T(p.vel), T(p.mass), T(np.arange(65536, dtype=np.int32)), eps2)
    torch.cuda.synchronize()
    a_ref = a_ref.cpu().numpy()
    rel = np.linalg.norm(acc1 - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
    assert np.sqrt(np.mean(rel ** 2)) < 1e-3
    interactions = st["accepted"] * 64 + st["opened_leaves"] * 16
    assert interactions < 0.1 * 65536 ** 2


def test_argument_errors(ctx):
    import paper_1409_5474_amd as nb
    import torch
    p = synth.plummer(100, 14)
    with pytest.raises(nb.NbodyError):
        ctx.tree_forces(T(p.pos), T(p.mass), -1.0, 0.5)
    with pytest.raises(nb.NbodyError):
        ctx.tree_forces(T(p.pos), T(p.mass), 1e-3, -0.1)
    with pytest.raises(nb.NbodyError):
        ctx.tree_forces(T(p.pos), T(p.mass), 1e-3, 0.5, n_crit=0)
    torch.cuda.synchronize()


@pytest.mark.parametrize("theta", [0.3, 0.6])
def test_mixed_precision_tree_forces(theta):
    # Same walk (the double one), float terms: the interaction set is the
    # oracle's and the forces are within float rounding of its.
    import paper_1409_5474_amd as nb
    from errors import vec_err
    p = synth.plummer(4000, 15)
    eps2 = 1e-4
    cm = nb.Context(0, "mixed")
    acc, pot, st = _gpu(cm, p.pos, p.mass, eps2, theta)
    cm.close()
    ra, rp, rst, t = _oracle(p.pos, p.mass, eps2, theta)
    assert st["accepted"] == sum(c for c, _, _ in rst)
    assert st["opened_leaves"] == sum(l for _, l, _ in rst)
    ea = vec_err(acc, ra, np.linalg.norm(ra, axis=1))
    ep = vec_err(pot, rp, np.abs(rp))
    assert ea["rms"] < 1e-6 and ea["normwise"] < 1e-6, ea
    assert ep["rms"] < 1e-6, ep


def _clustered(n, seed):
    """Nested clumps packed ever tighter: a deep octree."""
    rng = np.random.default_rng(seed)
    pos = rng.standard_normal((n, 3))
    m = n // 3
    for _ in range(7):
        pos[:m] = pos[:m] * 0.1 + 0.3
        m //= 2
    return pos, np.full(n, 1.0 / n)


@pytest.mark.parametrize("n_crit,theta", [(1, 0.5), (100, 0.5), (200, 0.0), (300, 0.7)])
def test_leaf_sizes_from_one_to_beyond_a_wavefront(ctx, n_crit, theta):
    # leaves of one particle (the deepest tree) and leaves far larger than the
    # 64 particles the kernel stages at a time
    p = synth.plummer(2500, 16)
    acc, pot, st = _gpu(ctx, p.pos, p.mass, 1e-4, theta, n_crit)
    ra, rp, rst, t = _oracle(p.pos, p.mass, 1e-4, theta, n_crit)
    assert st["accepted"] == sum(c for c, _, _ in rst)
    assert st["opened_leaves"] == sum(l for _, l, _ in rst)
    assert st["cells"] == len(t.cells)
    _close((acc, pot), (ra, rp), 1e-12, p.pos, p.mass, 1e-4)


@pytest.mark.parametrize("theta", [0.0, 0.6])
def test_deep_clustered_tree(ctx, theta):
    pos, mass = _clustered(3000, 17)
    acc, pot, st = _gpu(ctx, pos, mass, 1e-8, theta, 8)
    ra, rp, rst, t = _oracle(pos, mass, 1e-8, theta, 8)
    assert st["depth"] == max(c.level for c in t.cells) >= 10
    assert st["accepted"] == sum(c for c, _, _ in rst)
    assert st["opened_leaves"] == sum(l for _, l, _ in rst)
    _close((acc, pot), (ra, rp), 1e-12, pos, mass, 1e-8)


@pytest.mark.parametrize("n,seed", [(1, 1), (2047, 2), (2048, 3), (2049, 4), (100000, 5)])
def test_curve_order_is_the_oracles_lexsort(ctx, n, seed):
    # The library's radix sort against numpy's: identical keys and rows
    # (integer work, bit for bit), including ties (coincident particles).
    import torch
    pos = synth.plummer(n, seed).pos
    if n > 10:
        pos[n // 2: n // 2 + 7] = pos[3]  # equal keys: the order among them is the input order
    keys, idx = ctx.tree_keys(T(pos))
    torch.cuda.synchronize()
    lo, side = TR.box(pos)
    ref_keys = TR.hilbert_keys(TR.grid_coords(pos, lo, side))
    order = np.lexsort((np.arange(n), ref_keys))
    assert np.array_equal(idx.cpu().numpy(), order)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ref_keys[order].astype(np.uint64))


def test_tree_forces_replay_from_a_graph(ctx):
    # With stats off the evaluation reads nothing on the host, so it can be
    # captured; every replay (with other work and synchronisations between)
    # gives the eager bits.
    import torch
    p = synth.plummer(20000, 9)
    P, M = T(p.pos), T(p.mass)
    a0, f0, st = ctx.tree_forces(P, M, 1e-4, 0.5)          # eager, sizes the buffers
    assert st["cells"] > 1
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    acc = torch.empty_like(a0)
    pot = torch.empty_like(f0)
    with torch.cuda.stream(s):
        ctx.tree_forces(P, M, 1e-4, 0.5, acc=acc, pot=pot, stats=False)  # warm-up on the stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.tree_forces(P, M, 1e-4, 0.5, acc=acc, pot=pot, stats=False)
    torch.cuda.synchronize()
    for r in range(3):
        with torch.cuda.stream(s):
            acc.zero_()
            pot.zero_()
            g.replay()
        torch.cuda.synchronize()
        assert torch.equal(acc, a0) and torch.equal(pot, f0), r
        ctx.tree_forces(P, M, 1e-4, 0.7)                      # other eager work between replays
    ctx.set_stream(None)
    ctx.sync()
