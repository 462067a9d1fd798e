"""GPU parity of the sixth-order Hermite pieces against the CPU oracle,
through the C ABI: the snap force kernel (FP64 gate per particle), the
predictor, the corrector with its step criterion and levels, the start-up
levels, and whole block steps (eager and graph-replayed)."""
import numpy as np
import pytest

import oracle
from oracle import hermite6 as H6
import synth
from errors import check_fp64

pytestmark = pytest.mark.gpu
NAMES = ("acc", "jerk", "snap", "pot")


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


def _state(n, seed):
    p = synth.plummer(n, seed)
    acc_j = oracle.forces_f64(p.pos, p.vel, p.mass, 1e-3)[0]    # a physical acceleration field
    return p, acc_j


def _gpu6(ctx, p, acc_j, eps2, act):
    import torch
    a, j, s, pot = ctx.forces6(T(p.pos), T(p.vel), T(acc_j), T(p.mass), T(act.astype(np.int32)), eps2)
    torch.cuda.synchronize()
    return a.cpu().numpy(), j.cpu().numpy(), s.cpu().numpy(), pot.cpu().numpy()


@pytest.mark.parametrize("n,na,seed", [(1024, 1024, 1), (3001, 777, 7), (1, 1, 2), (300, 8, 3), (5000, 257, 4)])
def test_forces6_match_oracle(ctx, n, na, seed):
    p, acc_j = _state(n, seed)
    rng = np.random.default_rng(n)
    act = np.sort(rng.choice(n, na, replace=False)).astype(np.int32)
    if na > 3:
        act[2] = act[1]                                   # duplicates are computed independently
    eps2 = 1e-3
    ref = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, eps2, act)
    check_fp64(_gpu6(ctx, p, acc_j, eps2, act), ref, names=NAMES)


def test_forces6_unsoftened_with_a_coincident_pair(ctx):
    p, acc_j = _state(700, 9)
    p.pos[5] = p.pos[600]
    act = np.arange(0, 700, 3).astype(np.int32)
    ref = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, 0.0, act)
    assert ref["skipped"] >= 1
    check_fp64(_gpu6(ctx, p, acc_j, 0.0, act), ref, names=NAMES)


def test_forces6_acc_jerk_pot_agree_with_the_fourth_order_kernel(ctx):
    import torch
    p, acc_j = _state(2000, 5)
    act = T(np.arange(2000, dtype=np.int32))
    a6, j6, _, p6 = ctx.forces6(T(p.pos), T(p.vel), T(acc_j), T(p.mass), act, 1e-3)
    a4, j4, p4 = ctx.forces(T(p.pos), T(p.vel), T(p.mass), act, 1e-3)
    torch.cuda.synchronize()
    for x, y in ((a6, a4), (j6, j4), (p6, p4)):
        assert torch.linalg.norm(x - y) <= 1e-14 * torch.linalg.norm(y)


def test_predict6_matches_oracle(ctx):
    import torch
    rng = np.random.default_rng(11)
    n, ML, dt_max = 777, 20, 1.0 / 16
    x, v, a, j, s, c = rng.standard_normal((6, n, 3))
    t_tick = np.sort(rng.integers(0, 1 << ML, n)).astype(np.int64)
    t_next = int(t_tick.max()) + 12345
    dt_min = dt_max * 2.0 ** -ML
    out = [torch.empty((n, 3), dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.predict6(T(x), T(v), T(a), T(j), T(s), T(c), T(t_tick), t_next, dt_min, *out)
    torch.cuda.synchronize()
    ref = H6.predict(x, v, a, j, s, c, (t_next - t_tick) * dt_min)
    for got, r in zip(out, ref):
        np.testing.assert_allclose(got.cpu().numpy(), r, rtol=1e-13, atol=1e-15)


def test_correct6_and_levels_match_oracle(ctx):
    # A smooth acceleration history per particle (a quintic in time) gives
    # (a, j, s) at both ends of each particle's step; the corrector must
    # reproduce the oracle's positions, velocities, crackle and levels.
    import torch
    from oracle import hermite as H
    rng = np.random.default_rng(12)
    n, ML, dt_max, eta = 500, 20, 1.0 / 16, 0.15
    level = rng.integers(3, 12, n).astype(np.int32)
    h = dt_max * 2.0 ** -level.astype(np.float64)
    t0 = np.zeros(n, dtype=np.int64)
    # derivatives on the time scale of four steps, as a well-chosen level has
    tau = 4.0 * h[None, :, None]
    A = rng.standard_normal((6, n, 3)) * tau ** -np.arange(6.0)[:, None, None]
    fact = [1, 1, 2, 6, 24, 120]
    H1 = h[:, None]
    a0, j0, s0 = A[0], A[1], A[2]
    a1 = sum(A[k] * H1 ** k / fact[k] for k in range(6))
    j1 = sum(A[k] * H1 ** (k - 1) / fact[k - 1] for k in range(1, 6))
    s1 = sum(A[k] * H1 ** (k - 2) / fact[k - 2] for k in range(2, 6))
    x0, v0 = rng.standard_normal((2, n, 3))
    c_old = rng.standard_normal((n, 3))
    act = np.arange(n, dtype=np.int32)
    dev = [T(z) for z in (x0, v0, a0, j0, s0, c_old)]
    tt, lv = T(t0), T(level)
    clamps = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.correct6(T(act), T(a1), T(j1), T(s1), *dev, tt, lv, eta, dt_max, ML, clamps)
    torch.cuda.synchronize()
    c0, p0, q0 = H6.interpolate(a0, j0, s0, a1, j1, s1, h)
    x1, v1, c1, p1 = H6.correct(x0, v0, a0, j0, s0, c0, p0, q0, h)
    ds = H6.new_dt(a1, j1, s1, c1, p1, q0, eta, dt_max)
    t_new = t0 + np.left_shift(np.int64(1), (ML - level).astype(np.int64))
    lev, cl = H.new_level(level, ds, t_new, dt_max, ML)
    np.testing.assert_allclose(dev[0].cpu().numpy(), x1, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(dev[1].cpu().numpy(), v1, rtol=1e-13, atol=1e-14)
    np.testing.assert_array_equal(dev[2].cpu().numpy(), a1)
    np.testing.assert_array_equal(dev[3].cpu().numpy(), j1)
    np.testing.assert_array_equal(dev[4].cpu().numpy(), s1)
    # The crackle is a third derivative recovered from values at two times:
    # rounding in a1 - (a0 + j0 h + s0 h^2/2) is amplified by 1/h^3, so both
    # the GPU's closed form and the oracle's linear solve are held to the
    # exact crackle of the quintic within that conditioning bound.
    c_exact = A[3] + A[4] * H1 + A[5] * H1 ** 2 / 2
    M = np.maximum.reduce([np.abs(a0).max(1), np.abs(a1).max(1), (np.abs(j0) * H1).max(1),
                           (np.abs(s0) * H1 ** 2).max(1)])
    bound = 1000 * 2.0 ** -53 * M / h ** 3
    assert np.all(np.abs(c1 - c_exact).max(1) <= bound)
    assert np.all(np.abs(dev[5].cpu().numpy() - c_exact).max(1) <= bound)
    # and so the GPU's crackle against the oracle's, row by row
    assert np.all(np.abs(dev[5].cpu().numpy() - c1).max(1) <= 2 * bound)
    np.testing.assert_array_equal(tt.cpu().numpy(), t_new)
    np.testing.assert_array_equal(lv.cpu().numpy(), lev)
    assert int(clamps.item()) == int(cl.sum())


def test_startup6_levels_match_oracle(ctx):
    import torch
    p, acc_j = _state(1500, 13)
    r = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, 1e-3)
    lev = torch.zeros(1500, dtype=torch.int32, device="cuda")
    ctx.startup6(T(r["acc"]), T(r["jerk"]), T(r["snap"]), 0.02, 1.0 / 16, 24, lev)
    ref, _ = H6.startup_level(r["acc"], r["jerk"], r["snap"], 0.02, 1.0 / 16, 24)
    np.testing.assert_array_equal(lev.cpu().numpy(), ref)


@pytest.mark.parametrize("use_graph", [False, True])
def test_block_steps6_follow_the_oracle(use_graph):
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator6
    n, eps2, eta, eta_s, dt_max, ML = 512, 1e-3, 0.15, 0.01, 1.0 / 16, 24
    p = synth.plummer(n, 17)
    ctx = nb.Context(0, "fp64")
    bi = BlockIntegrator6(ctx, T(p.pos), T(p.vel), T(p.mass), eps2, eta, dt_max, ML, eta_s)
    st = H6.initialise(p.pos, p.vel, p.mass, eps2, eta, eta_s, dt_max, ML, H6.oracle_forces6(eps2))
    np.testing.assert_array_equal(bi.level.cpu().numpy(), st.level)
    bi.run_until(0.0625, graph_steps=8, use_graph=use_graph)
    H6.run_until(st, 0.0625, H6.oracle_forces6(eps2))
    torch.cuda.synchronize()
    assert bi.steps == st.steps
    np.testing.assert_array_equal(bi.level.cpu().numpy(), st.level)
    np.testing.assert_array_equal(bi.t_tick.cpu().numpy(), st.t)
    for got, ref in ((bi.pos, st.x), (bi.vel, st.v), (bi.acc, st.a), (bi.jerk, st.j)):
        d = np.abs(got.cpu().numpy() - ref).max()
        assert d <= 1e-10 * np.abs(ref).max(), d
    ctx.close()


def test_sixth_order_drift_is_far_below_fourth_order_at_equal_work():
    # Same Plummer model, same end time; the order-six run with about the
    # same number of force evaluations conserves energy far better.
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator, BlockIntegrator6
    p = synth.plummer(2048, 19)
    eps2 = 1e-4
    ctx = nb.Context(0, "fp64")
    b4 = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), eps2, 0.02, 1.0 / 16, 30)
    E0 = b4.energy()["E"]
    b4.run_until(0.125)
    d4 = abs(b4.energy()["E"] - E0) / abs(E0)
    b6 = BlockIntegrator6(ctx, T(p.pos), T(p.vel), T(p.mass), eps2, 0.4, 1.0 / 16, 30, 0.02)
    b6.run_until(0.125)
    d6 = abs(b6.energy()["E"] - E0) / abs(E0)
    print("drift 4th", d4, b4.steps, "6th", d6, b6.steps)
    assert d6 < 0.1 * d4, (d4, d6)
    ctx.close()


def test_checkpoint_resume6_is_bitwise(tmp_path):
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator6
    p = synth.plummer(700, 23)
    ctx = nb.Context(0, "fp64")
    args = (ctx, T(p.pos), T(p.vel), T(p.mass), 1e-3, 0.2, 1.0 / 16, 24, 0.01)
    straight = BlockIntegrator6(*args).run_until(0.125, graph_steps=8)
    half = BlockIntegrator6(*args).run_until(0.0625, graph_steps=8)
    path = tmp_path / "state6.npz"
    half.checkpoint(str(path))
    resumed = BlockIntegrator6.restore(ctx, str(path)).run_until(0.125, graph_steps=8)
    for k in ("pos", "vel", "acc", "jerk", "snap", "crackle", "t_tick", "level"):
        assert torch.equal(getattr(straight, k), getattr(resumed, k)), k
    ctx.close()


def test_forces6_full_size_sampled(ctx):
    # The snap kernel at the 262144-body Plummer workload's size, in the
    # launch the block steps use: 256 evenly spaced rows against the oracle,
    # element by element.  The j-accelerations (an input of the snap) are
    # the Plummer model's own field -x (|x|^2 + 1)^-3/2, so no input comes
    # from the library.
    n = 262144
    p = synth.plummer(n, 3)
    r2 = np.sum(p.pos ** 2, axis=1, keepdims=True)
    acc_j = -p.pos * (r2 + 1.0) ** -1.5
    act = np.linspace(0, n - 1, 256).astype(np.int32)
    eps2 = 2.0 ** -16
    ref = oracle.snap_ld(p.pos, p.vel, acc_j, p.mass, eps2, act)
    check_fp64(_gpu6(ctx, p, acc_j, eps2, act), ref, names=NAMES)
