"""GPU parity of the Hermite block-step kernels (predict, correct, start-up
levels, scheduler, energy, whole block steps, graph replay) and of the
batched and device-count force launches, against the CPU oracle; batches in
every precision and shape, with an unsoftened system among softened ones."""
import numpy as np
import pytest

import oracle
import synth
from errors import check_fp64, check_mixed
from oracle import hermite as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    import paper_1409_5474_amd as nbm
    return nbm


@pytest.fixture(scope="module")
def ctx(nb):
    c = nb.Context(0, "fp64")
    yield c
    c.close()


def T(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return (t.to(dtype) if dtype is not None else t).cuda()


def N(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rand_state(n, seed, max_level=20):
    rng = np.random.default_rng(seed)
    x, v, a, j = rng.standard_normal((4, n, 3))
    level = rng.integers(0, 8, n).astype(np.int32)
    # t_i a multiple of the particle's step, below the next common sync
    ticks = (np.int64(1) << (max_level - level.astype(np.int64)))
    t_tick = rng.integers(0, 4, n).astype(np.int64) * ticks
    return x, v, a, j, level, t_tick


def test_predict(ctx):
    ML, dt_max = 20, 1.0 / 16
    x, v, a, j, level, t_tick = _rand_state(1000, 1, ML)
    t_next = int((t_tick + (np.int64(1) << (ML - level.astype(np.int64)))).max())
    dt_min = dt_max * 2.0 ** -ML
    import torch
    pp = torch.empty((1000, 3), dtype=torch.float64, device="cuda"); vp = torch.empty_like(pp)
    ctx.predict(T(x), T(v), T(a), T(j), T(t_tick), t_next, dt_min, pp, vp)
    ex, ev = H.predict(x, v, a, j, (t_next - t_tick).astype(np.float64) * dt_min)
    np.testing.assert_allclose(N(pp), ex, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(N(vp), ev, rtol=1e-14, atol=1e-14)


def test_correct_and_levels(ctx):
    import torch
    ML, dt_max, eta = 24, 1.0 / 16, 0.01
    n = 3000
    rng = np.random.default_rng(2)
    x, v, a0, j0, level, t_tick = _rand_state(n, 2, ML)
    # forces at the end of the step: a smooth change plus noise of various sizes
    dtv = dt_max * 2.0 ** -level.astype(np.float64)
    scale = 10.0 ** rng.uniform(-3, 1, n)
    a1 = a0 + j0 * dtv[:, None] + scale[:, None] * rng.standard_normal((n, 3)) * dtv[:, None] ** 2
    j1 = j0 + scale[:, None] * rng.standard_normal((n, 3)) * dtv[:, None]
    act = np.sort(rng.choice(n, 1200, replace=False)).astype(np.int32)
    xp, vp = H.predict(x, v, a0, j0, dtv)
    # oracle
    a2, a3 = H.interpolate(a0[act], j0[act], a1[act], j1[act], dtv[act])
    ex, ev = H.correct(xp[act], vp[act], a2, a3, dtv[act])
    ds = H.aarseth_dt(a1[act], j1[act], a2, a3, dtv[act], eta, dt_max)
    t_new = t_tick[act] + (np.int64(1) << (ML - level[act].astype(np.int64)))
    elev, ecl = H.new_level(level[act], ds, t_new, dt_max, ML)
    # GPU
    g = dict(pos=T(x), vel=T(v), acc=T(a0), jerk=T(j0), t=T(t_tick), lev=T(level))
    clamp = torch.zeros(1, dtype=torch.int64, device="cuda")
    ctx.correct(T(act), T(xp), T(vp), T(a1[act]), T(j1[act]), g["pos"], g["vel"], g["acc"], g["jerk"], g["t"],
                g["lev"], eta, dt_max, ML, clamp)
    np.testing.assert_allclose(N(g["pos"])[act], ex, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(N(g["vel"])[act], ev, rtol=1e-13, atol=1e-13)
    assert np.array_equal(N(g["acc"])[act], a1[act]) and np.array_equal(N(g["jerk"])[act], j1[act])
    assert np.array_equal(N(g["t"])[act], t_new)
    gl = N(g["lev"])[act]
    # level decisions agree except where dt* sits on a power-of-two boundary to rounding
    assert np.mean(gl == elev) > 0.999, np.sum(gl != elev)
    assert int(N(clamp)[0]) == int(ecl.sum())
    # inactive rows untouched
    rest = np.setdiff1d(np.arange(n), act)
    assert np.array_equal(N(g["pos"])[rest], x[rest]) and np.array_equal(N(g["lev"])[rest], level[rest])


def test_startup_levels(ctx):
    import torch
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2000, 3)) * 10.0 ** rng.uniform(-2, 2, (2000, 1))
    j = rng.standard_normal((2000, 3)) * 10.0 ** rng.uniform(-2, 4, (2000, 1))
    j[5] = 0.0
    lev = torch.empty(2000, dtype=torch.int32, device="cuda")
    ctx.startup(T(a), T(j), 0.01, 1.0 / 16, 30, lev)
    ref, _ = H.startup_level(a, j, 0.01, 1.0 / 16, 30)
    assert np.array_equal(N(lev), ref)


@pytest.mark.parametrize("n", [1, 5, 1023, 1024, 1025, 70001])
def test_schedule_exact(ctx, n):
    import torch
    ML = 30
    rng = np.random.default_rng(n)
    level = rng.integers(0, 12, n).astype(np.int32)
    ticks = (np.int64(1) << (ML - level.astype(np.int64)))
    t_tick = rng.integers(0, 3, n).astype(np.int64) * ticks
    t_end = t_tick + ticks
    t_next = t_end.min()
    expect = np.nonzero(t_end == t_next)[0].astype(np.int32)
    active = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    sched = torch.zeros(4, dtype=torch.int64, device="cuda")
    ctx.schedule(T(t_tick), T(level), ML, active, sched)
    s = N(sched)
    assert s[0] == t_next and s[1] == expect.size
    assert np.array_equal(N(active)[:expect.size], expect)


def test_energy(ctx):
    import torch
    p = synth.plummer(5000, 4)
    r = oracle.forces_ld(p.pos, p.vel, p.mass, 1e-3)
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    ctx.energy(T(p.pos), T(p.vel), T(p.mass), T(r["pot"]), out)
    e = H.energy(p.pos, p.vel, p.mass, r["pot"])
    o = N(out)
    assert o[0] == pytest.approx(e["K"], rel=1e-13)
    assert o[1] == pytest.approx(e["W"], rel=1e-13)
    np.testing.assert_allclose(o[2:5], e["P"], atol=1e-15)
    np.testing.assert_allclose(o[5:8], e["L"], atol=1e-14)


class DeviceRun:
    """Block-step integration on the GPU through nb_block_step."""

    def __init__(self, ctx, p, eps2, eta, dt_max, max_level):
        import torch
        self.ctx, self.n = ctx, p.mass.shape[0]
        self.eps2, self.eta, self.dt_max, self.ML = eps2, eta, dt_max, max_level
        n = self.n
        f = lambda: torch.empty((n, 3), dtype=torch.float64, device="cuda")
        self.mass = T(p.mass)
        self.pos, self.vel, self.acc, self.jerk = T(p.pos), T(p.vel), f(), f()
        self.pos_p, self.vel_p, self.acc1, self.jerk1 = f(), f(), f(), f()
        self.pot1 = torch.empty(n, dtype=torch.float64, device="cuda")
        self.active = torch.empty(n, dtype=torch.int32, device="cuda")
        self.t = torch.zeros(n, dtype=torch.int64, device="cuda")
        self.lev = torch.empty(n, dtype=torch.int32, device="cuda")
        self.sched = torch.zeros(4, dtype=torch.int64, device="cuda")
        allact = torch.arange(n, dtype=torch.int32, device="cuda")
        ctx.forces(self.pos, self.vel, self.mass, allact, eps2, self.acc, self.jerk, self.pot1)
        ctx.startup(self.acc, self.jerk, eta, dt_max, max_level, self.lev)

    def step(self):
        self.ctx.block_step(self.n, self.eps2, self.eta, self.dt_max, self.ML, self.mass, self.pos, self.vel,
                            self.acc, self.jerk, self.t, self.lev, self.pos_p, self.vel_p, self.active, self.acc1,
                            self.jerk1, self.pot1, self.sched)


def _cpu_forces(eps2):
    def f(x, v, m, act):
        a, j, p, _ = oracle.forces_f64(x, v, m, eps2, act)
        return a, j, p
    return f


def test_block_steps_match_cpu_hermite(ctx):
    # Plummer N = 1024, eps = 0.01, eta = 0.02, block steps to t = 1/8.
    n, eps2, eta, dt_max, ML = 1024, 1e-4, 0.02, 1.0 / 16, 30
    p = synth.plummer(n, 1)
    st = H.initialise(p.pos, p.vel, p.mass, eps2, eta, dt_max, ML, _cpu_forces(eps2))
    g = DeviceRun(ctx, p, eps2, eta, dt_max, ML)
    assert np.array_equal(N(g.lev), st.level)
    end = int(round(0.125 / st.tick))
    hist_gpu = []
    while int(st.t.min()) < end:
        H.block_step(st, _cpu_forces(eps2))
        g.step()
        hist_gpu.append(int(N(g.sched)[1]))
    assert int(N(g.sched)[2]) == st.steps
    flips = sum(1 for a, b in zip(hist_gpu, st.n_active_hist) if a != b)
    assert flips == 0, flips
    assert np.array_equal(N(g.t), st.t) and np.array_equal(N(g.lev), st.level)
    dx = np.abs(N(g.pos) - st.x).max()
    assert dx < 1e-11, dx
    import torch
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    allact = torch.arange(n, dtype=torch.int32, device="cuda")
    _, _, pot = ctx.forces(g.pos, g.vel, g.mass, allact, eps2)
    ctx.energy(g.pos, g.vel, g.mass, pot, out)
    e_cpu = H.energy(st.x, st.v, st.m, oracle.forces_ld(st.x, st.v, st.m, eps2)["pot"])
    assert N(out)[0] + N(out)[1] == pytest.approx(e_cpu["E"], rel=1e-12)


def test_block_step_graph_replay_matches_eager(ctx):
    import torch
    n, eps2, eta, dt_max, ML = 2000, 1e-4, 0.02, 1.0 / 16, 30
    p = synth.plummer(n, 8)
    eager = DeviceRun(ctx, p, eps2, eta, dt_max, ML)
    graph_run = DeviceRun(ctx, p, eps2, eta, dt_max, ML)
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    with torch.cuda.stream(s):
        graph_run.step()          # eager warm-up: sizes the workspaces
        eager.step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        graph_run.step()
    torch.cuda.synchronize()
    for r in range(12):
        # the replay goes to the context's stream too: calls on one context
        # must not overlap on the device
        with torch.cuda.stream(s):
            g.replay()
            eager.step()
        torch.cuda.synchronize()
        for a, b in ((graph_run.pos, eager.pos), (graph_run.vel, eager.vel), (graph_run.t, eager.t),
                     (graph_run.lev, eager.lev), (graph_run.sched, eager.sched)):
            assert torch.equal(a, b), r
    ctx.set_stream(None)
    ctx.sync()  # raises if the work-queue counters were left non-zero


@pytest.mark.parametrize("prec,n", [("fp64", 20000), ("mixed", 20000), ("fp64", 65536), ("mixed", 65536)])
def test_devcount_matches_host_count(ctx, prec, n):
    # Bit for bit, with the shipped tuning table: at N = 65536 its regimes of
    # one shape share a device-count launch, which must still give each count
    # the j-split a host-count launch chooses.
    import torch
    ctx.set_precision(prec)
    p = synth.plummer(n, 12)
    P, V, M = T(p.pos), T(p.vel), T(p.mass)
    counts = (1, 3, 20, 100, 300, 1000, 3000, 9000, 20000, 40000, 65536)
    for na in [c for c in counts if c <= n]:
        act = T(np.sort(np.random.default_rng(na).choice(n, na, replace=False)).astype(np.int32))
        a1, j1, p1 = ctx.forces(P, V, M, act, 1e-3)
        cnt = torch.tensor([na], dtype=torch.int32, device="cuda")
        a2 = torch.empty((n, 3), dtype=torch.float64, device="cuda"); j2 = torch.empty_like(a2)
        p2 = torch.empty(n, dtype=torch.float64, device="cuda")
        act_full = torch.zeros(n, dtype=torch.int32, device="cuda"); act_full[:na] = act
        ctx.forces_devcount(P, V, M, act_full, cnt, n, 1e-3, a2, j2, p2)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2[:na]) and torch.equal(j1, j2[:na]) and torch.equal(p1, p2[:na]), na
    ctx.set_precision("fp64")


@pytest.mark.parametrize("shape", [None, (1, 0), (2, 0), (2, 4)], ids=["table", "sj1", "sj2", "lds2x4"])
@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_ds"])
def test_batch_matches_oracle(nb, prec, shape):
    # every batched kernel shape (default choice, the scalar j-path with one
    # or two i-particles per lane, the LDS layout) on its own context
    import torch
    ctx = nb.Context(0, prec)
    if shape is not None:
        ctx.tune_add_batch(prec, 1, 1, 2 ** 40, *shape)
        assert ctx.get_batch_launch(1, 500, 1000) == shape
    b = synth.cluster_batch(seed=4, n_clusters=24, n_min=64, n_max=3000)
    rng = np.random.default_rng(5)
    acts, aoff = [], [0]
    for c in range(24):
        lo, hi = b.offsets[c], b.offsets[c + 1]
        k = max(1, int((hi - lo) * rng.uniform(0.05, 1.0)))
        acts.append(np.sort(rng.choice(np.arange(lo, hi), k, replace=False)))
        aoff.append(aoff[-1] + k)
    act = np.concatenate(acts).astype(np.int32)
    na = act.size
    acc = torch.empty((na, 3), dtype=torch.float64, device="cuda"); jerk = torch.empty_like(acc)
    pot = torch.empty(na, dtype=torch.float64, device="cuda")
    ctx.forces_batch(b.offsets, b.eps2, T(b.pos), T(b.vel), T(b.mass), T(act), aoff, acc, jerk, pot)
    A, J, Pt = N(acc), N(jerk), N(pot)
    for c in range(24):
        lo, hi = b.offsets[c], b.offsets[c + 1]
        rows = slice(aoff[c], aoff[c + 1])
        ref = oracle.forces_ld(b.pos[lo:hi], b.vel[lo:hi], b.mass[lo:hi], b.eps2[c], act[rows] - lo)
        # element-wise, with the same gates as the single-system parity tests
        if prec == "fp64":
            check_fp64((A[rows], J[rows], Pt[rows]), ref)
        else:
            check_mixed((A[rows], J[rows], Pt[rows]), ref)
    ctx.close()


@pytest.mark.parametrize("prec,shape", [("fp64", None), ("fp64", (2, 1)), ("mixed", None), ("mixed", (2, 0)),
                                        ("mixed", (2, 4)), ("mixed_ds", None), ("mixed_ds", (2, 0))])
def test_batch_with_an_unsoftened_system(nb, prec, shape):
    # One system with eps2 = 0 among softened ones: the batch runs the masked
    # kernels (one i-particle per lane) whatever K the table gives, for the
    # all-active call and for a batched block step.
    import torch
    ctx = nb.Context(0, prec)
    if shape is not None:
        ctx.tune_add_batch(prec, 1, 1, 2 ** 40, *shape)
        ctx.tune_add_batch(prec, 2, 1, 2 ** 40, *shape)
    b = synth.cluster_batch(seed=6, n_clusters=5, n_min=300, n_max=4000)
    eps2 = b.eps2.copy()
    eps2[2] = 0.0
    n = int(b.offsets[-1])
    act = np.arange(n, dtype=np.int32)
    acc = torch.empty((n, 3), dtype=torch.float64, device="cuda"); jerk = torch.empty_like(acc)
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.forces_batch(b.offsets, eps2, T(b.pos), T(b.vel), T(b.mass), T(act), b.offsets, acc, jerk, pot)
    A, J, Pt = N(acc), N(jerk), N(pot)
    for c in range(5):
        lo, hi = b.offsets[c], b.offsets[c + 1]
        ref = oracle.forces_ld(b.pos[lo:hi], b.vel[lo:hi], b.mass[lo:hi], eps2[c], act[lo:hi] - lo)
        res = (A[lo:hi], J[lo:hi], Pt[lo:hi])
        if prec == "fp64":
            check_fp64(res, ref)
        elif eps2[c] > 0:
            check_mixed(res, ref)
        else:
            # unsoftened: a row's float rounding is bounded by its terms'
            # magnitudes (the single-system unsoftened gate)
            for name, got in zip(("acc", "jerk", "pot"), res):
                err = np.abs(got - ref[name]) if got.ndim == 1 else np.linalg.norm(got - ref[name], axis=1)
                assert (err <= 64 * 2.0 ** -24 * ref["abs_" + name]).all(), name
    # a batched block step over the same systems runs too
    from paper_1409_5474_amd.integrator import BlockIntegrator
    bi = BlockIntegrator(ctx, T(b.pos), T(b.vel), T(b.mass), eps2, 0.02, 1.0 / 16, 30, offsets=b.offsets)
    for _ in range(3):
        bi.step()
    ctx.sync()
    assert bi.steps == 3 and torch.isfinite(bi.pos).all()
    ctx.close()


@pytest.mark.parametrize("shape", [(1, 4), (2, 1), (1, 16)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_per_cluster_calls_bit_for_bit(nb, prec, shape):
    # In the LDS layout the batch cuts each system's j-range with the common
    # chunk length J = ceil(work / (IB x 8 x CUs) / T) x T (work = sum over
    # systems of the i-slots x j) into S_c = min(max(1, ceil(nj/J)), ceil(nj/T))
    # chunks; each cluster computed alone with the same (K, L, S_c) gives the
    # same bits, its sums being formed in the same order.
    import math
    import torch
    K, L = shape
    ctx = nb.Context(0, prec)
    ctx.tune_add_batch(prec, 1, 1, 2 ** 40, K, L)
    b = synth.cluster_batch(seed=12, n_clusters=6, n_min=300, n_max=6000)
    n = int(b.offsets[-1])
    act = np.arange(n, dtype=np.int32)
    acc = torch.empty((n, 3), dtype=torch.float64, device="cuda"); jerk = torch.empty_like(acc)
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.forces_batch(b.offsets, b.eps2, T(b.pos), T(b.vel), T(b.mass), T(act), b.offsets, acc, jerk, pot)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    IB, tile = (256 // L) * K, 256
    sizes = np.diff(b.offsets)
    work = float(sum(-(-int(s) // IB) * IB * int(s) for s in sizes))
    J = max(tile, math.ceil(work / (IB * 8.0 * cus) / tile) * tile)
    splits = []
    for c, nj in enumerate(sizes):
        nj = int(nj)
        S = max(1, min(-(-nj // J), -(-nj // tile)))
        splits.append(S)
        lo, hi = b.offsets[c], b.offsets[c + 1]
        ctx.set_launch(K, L, S)
        a1, j1, p1 = ctx.forces(T(b.pos[lo:hi]), T(b.vel[lo:hi]), T(b.mass[lo:hi]),
                                T(np.arange(nj, dtype=np.int32)), float(b.eps2[c]))
        torch.cuda.synchronize()
        assert torch.equal(a1, acc[lo:hi]) and torch.equal(j1, jerk[lo:hi]) and torch.equal(p1, pot[lo:hi]), (c, S)
    assert max(splits) > 1   # the case exercises the chunk sums
    ctx.close()
