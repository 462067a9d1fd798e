"""GPU integrator driver: graph replay equals eager stepping; block steps
of a single system and of a batch of independent systems follow the CPU
oracle's Hermite runs (per system) with no level flips, unsoftened too (a
two-body orbit); empty systems and systems without active rows leave a
batch's bits unchanged; checkpoints resume bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from errors import check_mixed
from oracle import hermite as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1409_5474_amd as nb
    c = nb.Context(0, "fp64")
    yield c
    c.close()


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def N(t):
    return t.cpu().numpy()


def _cpu_run(p, eps2, eta, dt_max, ML, t_end):
    def f(x, v, m, act):
        a, j, ph, _ = oracle.forces_f64(x, v, m, eps2, act)
        return a, j, ph
    st = H.initialise(p.pos, p.vel, p.mass, eps2, eta, dt_max, ML, f)
    H.run_until(st, t_end, f)
    return st


def test_single_system_graph_equals_eager_and_oracle(ctx):
    from paper_1409_5474_amd.integrator import BlockIntegrator
    n, eps2, eta, dt_max, ML = 1024, 1e-4, 0.02, 1.0 / 16, 30
    p = synth.plummer(n, 1)
    g = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), eps2, eta, dt_max, ML).run_until(0.125, graph_steps=16)
    e = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), eps2, eta, dt_max, ML).run_until(0.125,
                                                                                             use_graph=False)
    import torch
    assert torch.equal(g.pos, e.pos) and torch.equal(g.vel, e.vel) and torch.equal(g.level, e.level)
    assert g.steps == e.steps
    st = _cpu_run(p, eps2, eta, dt_max, ML, 0.125)
    assert g.steps == st.steps
    assert np.array_equal(g.level.cpu().numpy(), st.level)
    assert np.abs(g.pos.cpu().numpy() - st.x).max() < 1e-11
    assert g.time == 0.125


@pytest.mark.parametrize("shape", [None, (1, 0), (2, 0)], ids=["table", "sj1", "sj2"])
def test_batch_block_steps_follow_per_system_oracle(shape):
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    ctx = nb.Context(0, "fp64")
    if shape is not None:
        ctx.tune_add_batch("fp64", 2, 1, 2 ** 40, *shape)
    b = synth.cluster_batch(seed=4, n_clusters=10, n_min=64, n_max=1500)
    eta, dt_max, ML, t_end = 0.02, 1.0 / 16, 30, 0.0625
    bi = BlockIntegrator(ctx, T(b.pos), T(b.vel), T(b.mass), b.eps2, eta, dt_max, ML, offsets=b.offsets)
    bi.run_until(t_end, graph_steps=8)
    ev = BlockIntegrator(ctx, T(b.pos), T(b.vel), T(b.mass), b.eps2, eta, dt_max, ML, offsets=b.offsets)
    ev.run_until(t_end, use_graph=False)
    assert torch.equal(bi.pos, ev.pos) and torch.equal(bi.level, ev.level)
    X, L = bi.pos.cpu().numpy(), bi.level.cpu().numpy()
    evals = 0
    for c in range(10):
        lo, hi = b.offsets[c], b.offsets[c + 1]
        sub = synth.Particles(b.pos[lo:hi], b.vel[lo:hi], b.mass[lo:hi])
        st = _cpu_run(sub, b.eps2[c], eta, dt_max, ML, t_end)
        assert np.array_equal(L[lo:hi], st.level), c
        assert np.abs(X[lo:hi] - st.x).max() < 1e-11, c
        evals += st.force_evals - (hi - lo)
    # every system's particles advanced exactly as in its own run; the global
    # block count is at least the largest per-system count
    assert bi.steps >= 1
    assert int(bi.t_tick.min().item()) * bi.tick == t_end
    ctx.sync()
    ctx.close()


@pytest.mark.parametrize("batch", [False, True])
def test_checkpoint_resume_is_bitwise(ctx, tmp_path, batch):
    import torch
    from paper_1409_5474_amd.integrator import BlockIntegrator
    eta, dt_max, ML = 0.02, 1.0 / 16, 30
    if batch:
        b = synth.cluster_batch(seed=4, n_clusters=6, n_min=64, n_max=900)
        args = (T(b.pos), T(b.vel), T(b.mass), b.eps2)
        kw = dict(offsets=b.offsets)
    else:
        p = synth.plummer(1500, 13)
        args = (T(p.pos), T(p.vel), T(p.mass), 1e-4)
        kw = {}
    straight = BlockIntegrator(ctx, *args, eta, dt_max, ML, **kw).run_until(0.125, graph_steps=8)
    half = BlockIntegrator(ctx, *args, eta, dt_max, ML, **kw).run_until(0.0625, graph_steps=8)
    path = tmp_path / "state.npz"
    half.checkpoint(str(path))
    resumed = BlockIntegrator.restore(ctx, str(path)).run_until(0.125, graph_steps=8)
    for k in ("pos", "vel", "acc", "jerk", "t_tick", "level"):
        assert torch.equal(getattr(straight, k), getattr(resumed, k)), k
    assert straight.steps == resumed.steps


def test_one_graph_serves_every_stop_time(ctx):
    # The stop tick lives in device memory: the graph captured for the first
    # stop time replays unchanged for the next ones, and matches eager steps.
    import torch
    from paper_1409_5474_amd.integrator import BlockIntegrator
    p = synth.plummer(1200, 21)
    args = (T(p.pos), T(p.vel), T(p.mass), 1e-4, 0.02, 1.0 / 16, 30)
    g = BlockIntegrator(ctx, *args)
    e = BlockIntegrator(ctx, *args)
    for t_end in (0.0625, 0.125, 0.1875):
        g.run_until(t_end, graph_steps=8, use_graph=True)
        e.run_until(t_end, graph_steps=8, use_graph=False)
        assert int(g.t_tick.min().item()) * g.tick == t_end
    assert len(g._graphs) == 1
    for k in ("pos", "vel", "acc", "jerk", "t_tick", "level"):
        assert torch.equal(getattr(g, k), getattr(e, k)), k
    assert g.steps == e.steps


def test_run_until_logs_every_synchronisation_time(ctx):
    # log(diagnostics()) at t = dt_max, 2 dt_max, ... and the same end state
    # as a run without stops (the stop tick only ends graphs, steps are equal)
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    p = synth.plummer(2048, 51)
    a = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), 1e-3, 0.02, 1.0 / 32, 20)
    b = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), 1e-3, 0.02, 1.0 / 32, 20)
    rec = []
    a.run_until(1.0 / 8, log=rec.append)
    b.run_until(1.0 / 8)
    assert [r["t"] for r in rec] == [k / 32 for k in range(1, 5)]
    assert rec[-1]["steps"] == b.steps
    import torch
    assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
    for r in rec:
        assert r["dE_rel"] < 1e-4 and 0.5 < r["virial"] < 1.5
        assert set(r) >= {"t", "steps", "clamps", "E", "K", "W", "dE_rel", "P", "L", "virial"}
    # the drift is measured from the energy at t = 0, so the first stop
    # already shows the drift of the first dt_max
    assert rec[0]["dE_rel"] > 0.0
    assert rec[0]["dE_rel"] == abs(rec[0]["E"] - a.E0) / abs(a.E0)


def test_run_until_rejects_a_time_between_synchronisation_times(ctx, tmp_path):
    # t = 0.1 is a whole number of ticks but not a multiple of dt_max = 1/16:
    # with or without a log the call refuses instead of stopping early
    from paper_1409_5474_amd.integrator import BlockIntegrator
    p = synth.plummer(256, 52)
    a = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), 1e-3, 0.02, 1.0 / 16, 20)
    t0 = a.t_tick.clone()
    for log in (None, lambda r: None):
        with pytest.raises(ValueError):
            a.run_until(0.0625 + 2.0 ** -10, log=log)
    assert bool((a.t_tick == t0).all())
    # E0 survives a checkpoint
    a.run_until(0.0625)
    path = tmp_path / "st.npz"
    a.checkpoint(str(path))
    b = BlockIntegrator.restore(ctx, str(path))
    assert b.E0 == a.E0


def test_graph_capture_keeps_the_context_stream(ctx):
    # a context built on an explicit stream stays on it after run_until
    # captured its graph on a side stream
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    s = torch.cuda.Stream()
    c2 = nb.Context(0, "fp64", stream=s)
    p = synth.plummer(512, 53)
    with torch.cuda.stream(s):
        a = BlockIntegrator(c2, T(p.pos), T(p.vel), T(p.mass), 1e-3, 0.02, 1.0 / 16, 20)
        a.run_until(0.0625, graph_steps=4, use_graph=True)
    assert c2.stream is s
    torch.cuda.synchronize()
    c2.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_unsoftened_kepler_orbit_follows_the_oracle(use_graph):
    # eps2 = 0 runs the masked kernels in every block-step launch: an
    # eccentric two-body orbit (M = 1, a = 1, e = 0.5, from apocentre) over
    # one period, against the CPU oracle's block-step run with the same
    # levels, and its energy against the closed form -m1 m2 / (2 a) = -1/8.
    import types
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    e, eta, dt_max, ML, t_end = 0.5, 0.01, 1.0 / 16, 30, 6.3125
    r_apo = 1.0 + e
    v_rel = np.sqrt((1.0 - e) / (1.0 + e))
    pos = np.array([[-r_apo / 2, 0.0, 0.0], [r_apo / 2, 0.0, 0.0]])
    vel = np.array([[0.0, -v_rel / 2, 0.0], [0.0, v_rel / 2, 0.0]])
    mass = np.array([0.5, 0.5])
    ctx = nb.Context(0, "fp64")
    g = BlockIntegrator(ctx, T(pos), T(vel), T(mass), 0.0, eta, dt_max, ML).run_until(t_end, graph_steps=16,
                                                                                     use_graph=use_graph)
    p = types.SimpleNamespace(pos=pos, vel=vel, mass=mass)
    st = _cpu_run(p, 0.0, eta, dt_max, ML, t_end)
    assert g.steps == st.steps
    assert np.array_equal(g.level.cpu().numpy(), st.level)
    assert np.abs(g.pos.cpu().numpy() - st.x).max() < 1e-10
    E = g.energy()["E"]
    assert abs(E - (-0.125)) < 1e-6
    ctx.sync()
    ctx.close()


@pytest.mark.parametrize("shape", [(1, 0), (1, 16)], ids=["sj1", "lds1x16"])
def test_batch_with_empty_systems_and_inactive_systems(shape):
    # Empty systems (first, between and last) add no work, so with one shape
    # forced the batch gives the same bits as the batch without them: the
    # all-active call (one system also with no active rows there) and
    # graph-replayed block steps.
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    b = synth.cluster_batch(seed=9, n_clusters=3, n_min=200, n_max=1500)
    sizes = np.diff(b.offsets)
    full = np.array([0, 0, sizes[0], sizes[0], sizes[0] + sizes[1], sizes[:3].sum(), sizes[:3].sum()], dtype=np.int64)
    eps_full = np.array([1e-3, b.eps2[0], 2e-3, b.eps2[1], b.eps2[2], 5e-4])
    ctx = nb.Context(0, "mixed")
    for kind in (1, 2):
        ctx.tune_add_batch("mixed", kind, 1, 2 ** 40, *shape)
    n = int(b.offsets[-1])
    # all-active call, system 2 of the compact batch without active rows
    act = np.concatenate([np.arange(0, sizes[0]), np.arange(sizes[0] + sizes[1], n)]).astype(np.int32)
    act_off = np.array([0, sizes[0], sizes[0], act.size], dtype=np.int64)
    act_off_full = np.array([0, 0, sizes[0], sizes[0], sizes[0], act.size, act.size], dtype=np.int64)
    outs = []
    for offs, eps, aoff in ((b.offsets, b.eps2, act_off), (full, eps_full, act_off_full)):
        acc = torch.empty((act.size, 3), dtype=torch.float64, device="cuda"); jerk = torch.empty_like(acc)
        pot = torch.empty(act.size, dtype=torch.float64, device="cuda")
        ctx.forces_batch(offs, eps, T(b.pos), T(b.vel), T(b.mass), T(act), aoff, acc, jerk, pot)
        outs.append((acc, jerk, pot))
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(*outs))
    for c, rows in ((0, slice(0, sizes[0])), (2, slice(sizes[0], act.size))):
        lo, hi = b.offsets[c], b.offsets[c + 1]
        ref = oracle.forces_ld(b.pos[lo:hi], b.vel[lo:hi], b.mass[lo:hi], b.eps2[c], act[rows] - lo)
        check_mixed(tuple(N(o)[rows] for o in outs[0]), ref)
    # block steps
    runs = []
    for offs, eps in ((b.offsets, b.eps2), (full, eps_full)):
        bi = BlockIntegrator(ctx, T(b.pos), T(b.vel), T(b.mass), eps, 0.02, 1.0 / 16, 30, offsets=offs)
        bi.run_until(1.0 / 16, graph_steps=8)
        runs.append(bi)
    ctx.sync()
    assert runs[0].steps == runs[1].steps > 0
    for k in ("pos", "vel", "t_tick", "level"):
        assert torch.equal(getattr(runs[0], k), getattr(runs[1], k)), k
    ctx.close()
