"""GPU parity of the Hamiltonian-split pieces against the CPU oracle, through
the C ABI: forces on a separate i-set (every precision and launch shape),
the kick and kick-drift passes (bit-exact), and whole bridge steps of a
cluster inside a galaxy."""
import numpy as np
import pytest

import oracle
from oracle import bridge as OB
import synth
from errors import check_fp64, check_mixed

pytestmark = pytest.mark.gpu
PRECS = ["fp64", "mixed", "mixed_ds"]


def T(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.fixture(scope="module")
def ctx():
    import paper_1409_5474_amd as nb
    c = nb.Context(0, "fp64")
    yield c
    c.close()


def _sets(nj, ni, seed):
    pj = synth.plummer(nj, seed)
    pi = synth.plummer(ni, seed + 100)
    # the receivers sit inside and around the field set, some of them far out
    xi = pi.pos * 0.7 + np.array([0.2, -0.1, 0.05])
    return pj, xi, pi.vel


def _ref(pj, xi, vi, eps2, rows):
    nj, ni = pj.mass.size, xi.shape[0]
    pos = np.concatenate([pj.pos, xi])
    vel = np.concatenate([pj.vel, vi])
    mass = np.concatenate([pj.mass, np.zeros(ni)])
    return oracle.forces_ld(pos, vel, mass, eps2, (nj + rows).astype(np.int32))


def _run(ctx, prec, pj, xi, vi, eps2, rows, launch=None):
    import torch
    ctx.set_precision(prec)
    ctx.set_launch(*(launch or (0,)))
    try:
        acc, jerk, pot = ctx.forces_ij(T(pj.pos), T(pj.vel), T(pj.mass), T(xi), T(vi), T(rows.astype(np.int32)), eps2)
        torch.cuda.synchronize()
    finally:
        ctx.set_launch(0)
    return acc.cpu().numpy(), jerk.cpu().numpy(), pot.cpu().numpy()


def _check(prec, res, ref):
    if prec == "fp64":
        check_fp64(res, ref)
    else:
        check_mixed(res, ref)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nj,ni,na", [(1000, 300, 300), (3001, 777, 500), (1, 5, 5), (300, 1, 1), (257, 4000, 1234)])
def test_forces_ij_matches_oracle(ctx, prec, nj, ni, na):
    pj, xi, vi = _sets(nj, ni, 3)
    rng = np.random.default_rng(nj + ni)
    rows = np.sort(rng.choice(ni, na, replace=False))
    if na > 2:
        rows[1] = rows[0]                       # a duplicate row is computed twice
    eps2 = 1e-3
    _check(prec, _run(ctx, prec, pj, xi, vi, eps2, rows), _ref(pj, xi, vi, eps2, rows))


LAUNCHES = [(1, 1, 1), (2, 1, 3), (1, 16, 2), (1, 256, 1), (1, 0, 1), (2, 0, 3), (3, 0, 2), (2, -1, 3)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("launch", LAUNCHES)
def test_forces_ij_every_launch_shape(ctx, prec, launch):
    pj, xi, vi = _sets(2049, 700, 5)
    rows = np.arange(0, 700, 2)
    eps2 = 4e-4
    _check(prec, _run(ctx, prec, pj, xi, vi, eps2, rows, launch), _ref(pj, xi, vi, eps2, rows))


@pytest.mark.parametrize("prec", PRECS)
def test_forces_ij_unsoftened_coincident_pair_contributes_nothing(ctx, prec):
    pj, xi, vi = _sets(600, 50, 9)
    xi[7] = pj.pos[123]                          # a receiver on top of a field particle
    rows = np.arange(50)
    ref = _ref(pj, xi, vi, 0.0, rows)
    assert ref["skipped"] == 1
    _check(prec, _run(ctx, prec, pj, xi, vi, 0.0, rows), ref)


def test_forces_ij_equals_forces_with_massless_receivers(ctx):
    # The same sums through nbody_forces on the concatenated set, receivers
    # given mass zero: the two calls agree to rounding.
    import torch
    pj, xi, vi = _sets(1500, 400, 11)
    rows = np.arange(400)
    ctx.set_precision("fp64")
    a1, j1, p1 = ctx.forces_ij(T(pj.pos), T(pj.vel), T(pj.mass), T(xi), T(vi), T(rows.astype(np.int32)), 1e-3)
    pos = T(np.concatenate([pj.pos, xi])); vel = T(np.concatenate([pj.vel, vi]))
    mass = T(np.concatenate([pj.mass, np.zeros(400)]))
    a2, j2, p2 = ctx.forces(pos, vel, mass, T((1500 + rows).astype(np.int32)), 1e-3)
    torch.cuda.synchronize()
    for x, y in ((a1, a2), (j1, j2), (p1, p2)):
        assert torch.linalg.norm(x - y) <= 1e-14 * torch.linalg.norm(y)


def test_forces_ij_argument_errors(ctx):
    import torch
    import paper_1409_5474_amd as nb
    pj, xi, vi = _sets(100, 10, 1)
    rows = T(np.arange(10, dtype=np.int32))
    lib = nb.library()
    P = lambda t: None if t is None else __import__("ctypes").c_void_p(t.data_ptr())
    xj, vj, mj, xi_, vi_ = T(pj.pos), T(pj.vel), T(pj.mass), T(xi), T(vi)
    out = [torch.zeros((10, 3), dtype=torch.float64, device="cuda") for _ in range(2)]
    pot = torch.zeros(10, dtype=torch.float64, device="cuda")
    h = ctx.handle
    assert lib.nbody_forces_ij(h, P(xj), P(vj), P(mj), 100, None, P(vi_), 10, P(rows), 10, 1e-3,
                               P(out[0]), P(out[1]), P(pot)) == -1
    assert lib.nbody_forces_ij(h, P(xj), P(vj), P(mj), 100, P(xi_), P(vi_), 0, P(rows), 10, 1e-3,
                               P(out[0]), P(out[1]), P(pot)) == -1
    assert lib.nbody_forces_ij(h, P(xj), P(vj), P(mj), 0, P(xi_), P(vi_), 10, P(rows), 10, 1e-3,
                               P(out[0]), P(out[1]), P(pot)) == -1
    assert lib.nbody_forces_ij(h, P(xj), P(vj), P(mj), 100, P(xi_), P(vi_), 10, P(rows), 10, -1.0,
                               P(out[0]), P(out[1]), P(pot)) == -1
    # n_active = 0 is a no-op
    assert lib.nbody_forces_ij(h, P(xj), P(vj), P(mj), 100, None, None, 0, None, 0, 1e-3, None, None, None) == 0
    torch.cuda.synchronize()
    assert float(pot.abs().sum()) == 0.0


@pytest.mark.parametrize("n", [1, 5, 1000, 100003])
def test_kick_and_kick_drift_are_bit_exact(ctx, n):
    import torch
    rng = np.random.default_rng(n)
    x, v, a = rng.standard_normal((3, n, 3))
    h, hk = 0.0371, -0.01855
    X, V, A = T(x), T(v), T(a)
    ctx.kick(V, A, h)
    torch.cuda.synchronize()
    v1 = v + h * a
    np.testing.assert_array_equal(V.cpu().numpy(), v1)
    ctx.kick_drift(X, V, A, hk, h)
    torch.cuda.synchronize()
    v2 = v1 + hk * a
    np.testing.assert_array_equal(V.cpu().numpy(), v2)
    np.testing.assert_array_equal(X.cpu().numpy(), x + h * v2)


def _cluster_in_galaxy(n=600, n_c=40, seed=21, m_bh=0.02):
    p = synth.plummer(n, seed)
    order = np.argsort(np.linalg.norm(p.pos, axis=1), kind="stable")
    c, g = np.sort(order[:n_c]), np.sort(order[n_c:])
    mass = p.mass.copy()
    mass[c[np.argmin(np.linalg.norm(p.pos[c], axis=1))]] = m_bh
    return p, mass, g, c


@pytest.mark.parametrize("n_sub", [1, 3])
def test_bridge_steps_follow_the_oracle(n_sub):
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.bridge import Bridge
    p, mass, g, c = _cluster_in_galaxy()
    eps2_g, eps2_c, eps2_gc, dt, eta, ML = 1e-3, 1e-4, 5e-4, 1.0 / 64, 0.01, 20
    ctx = nb.Context(0, "fp64")
    br = Bridge(ctx, ctx, T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]),
                eps2_g, eps2_c, eps2_gc, dt, n_sub=n_sub, eta=eta, max_level=ML)
    st = OB.initialise(p.pos[g], p.vel[g], mass[g], p.pos[c], p.vel[c], mass[c], eps2_g, eps2_c, eps2_gc, dt,
                       n_sub=n_sub, eta=eta, max_level=ML)
    E0, E0_ref = br.energy()["E"], OB.energy(st)["E"]
    assert abs(E0 - E0_ref) <= 1e-13 * abs(E0_ref)
    for _ in range(6):
        br.step()
        OB.step(st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(br.cluster.level.cpu().numpy(), st.cluster.level)
    assert br.cluster.steps == st.cluster.steps
    for got, ref in ((br.xg, st.xg), (br.vg, st.vg), (br.cluster.pos, st.cluster.x), (br.cluster.vel, st.cluster.v)):
        d = np.abs(got.cpu().numpy() - ref).max()
        assert d <= 1e-11 * np.abs(ref).max(), d
    E1, E1_ref = br.energy()["E"], OB.energy(st)["E"]
    assert abs(E1 - E1_ref) <= 1e-12 * abs(E1_ref)
    assert abs(E1 - E0) <= 1e-4 * abs(E0)
    ctx.close()


def test_bridge_mixed_field_stays_close_to_fp64():
    # The cheap configuration: mixed precision for the galaxy and the cross
    # field, FP64 for the cluster; after a few steps it differs from the all-FP64
    # run by far less than the split error itself.
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.bridge import Bridge
    p, mass, g, c = _cluster_in_galaxy(n=2000, n_c=60, seed=4)
    args = (T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]), 1e-3, 1e-4, 5e-4, 1.0 / 64)
    c64, cmx = nb.Context(0, "fp64"), nb.Context(0, "mixed")
    ref = Bridge(c64, c64, *args).run(4)
    mix = Bridge(c64, cmx, *args).run(4)
    torch.cuda.synchronize()
    dx = float((mix.xg - ref.xg).abs().max())
    assert dx < 1e-6, dx
    assert abs(mix.energy()["E"] - ref.energy()["E"]) < 1e-6 * abs(ref.energy()["E"])
    c64.close(); cmx.close()


def test_bridge_with_the_tree_as_field_solver_follows_the_oracle():
    # The paper's hybrid: the field subsystem advanced with the tree code.
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.bridge import Bridge
    p, mass, g, c = _cluster_in_galaxy(n=1500, n_c=40, seed=31)
    eps2_g, eps2_c, eps2_gc, dt, eta, ML, theta = 1e-3, 1e-4, 5e-4, 1.0 / 64, 0.01, 20, 0.5
    ctx = nb.Context(0, "fp64")
    br = Bridge(ctx, ctx, T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]),
                eps2_g, eps2_c, eps2_gc, dt, eta=eta, max_level=ML, field="tree", theta=theta)
    st = OB.initialise(p.pos[g], p.vel[g], mass[g], p.pos[c], p.vel[c], mass[c], eps2_g, eps2_c, eps2_gc, dt,
                       eta=eta, max_level=ML, field=OB.tree_field(eps2_g, theta))
    for _ in range(3):
        br.step()
        OB.step(st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(br.cluster.level.cpu().numpy(), st.cluster.level)
    for got, ref in ((br.xg, st.xg), (br.vg, st.vg), (br.cluster.pos, st.cluster.x)):
        d = np.abs(got.cpu().numpy() - ref).max()
        assert d <= 1e-11 * np.abs(ref).max(), d
    ctx.close()


def test_bridge_with_the_tree_giving_the_cross_field_follows_the_oracle():
    # Each subsystem's solver gives the field it exerts: g's tree code (over
    # [g | c] with c massless) gives the field of g on c, the direct sum over
    # c the field of c on g.
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.bridge import Bridge
    p, mass, g, c = _cluster_in_galaxy(n=1500, n_c=40, seed=32)
    eps2_g, eps2_c, dt, eta, ML, theta = 1e-3, 1e-4, 1.0 / 64, 0.01, 20, 0.5
    ctx = nb.Context(0, "fp64")
    with pytest.raises(ValueError):
        Bridge(ctx, ctx, T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]),
               eps2_g, eps2_c, 2 * eps2_g, dt, field="tree", cross="tree")
    br = Bridge(ctx, ctx, T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]),
                eps2_g, eps2_c, eps2_g, dt, eta=eta, max_level=ML, field="tree", theta=theta, cross="tree")
    st = OB.initialise(p.pos[g], p.vel[g], mass[g], p.pos[c], p.vel[c], mass[c], eps2_g, eps2_c, eps2_g, dt,
                       eta=eta, max_level=ML, field=OB.tree_field(eps2_g, theta), cross="tree", theta=theta)
    for _ in range(3):
        br.step()
        OB.step(st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(br.cluster.level.cpu().numpy(), st.cluster.level)
    for got, ref in ((br.xg, st.xg), (br.vg, st.vg), (br.cluster.pos, st.cluster.x), (br.cluster.vel, st.cluster.v)):
        d = np.abs(got.cpu().numpy() - ref).max()
        assert d <= 1e-11 * np.abs(ref).max(), d
    ctx.close()


def test_bridge_graph_replay_equals_eager():
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.bridge import Bridge
    p, mass, g, c = _cluster_in_galaxy(n=800, n_c=40, seed=41)
    ctx = nb.Context(0, "fp64")
    args = (T(p.pos[g]), T(p.vel[g]), T(mass[g]), T(p.pos[c]), T(p.vel[c]), T(mass[c]), 1e-3, 1e-4, 5e-4, 1.0 / 64)
    a = Bridge(ctx, ctx, *args).run(4, use_graph=True)
    b = Bridge(ctx, ctx, *args).run(4, use_graph=False)
    torch.cuda.synchronize()
    assert len(a.cluster._graphs) == 1
    for x, y in ((a.xg, b.xg), (a.vg, b.vg), (a.cluster.pos, b.cluster.pos), (a.cluster.vel, b.cluster.vel)):
        assert torch.equal(x, y)
    ctx.close()
