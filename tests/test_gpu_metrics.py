"""Run-time diagnostics on the GPU: NB_LOG's error and launch lines, the
phase timing of eager block steps, and the integrator's per-step records
(active counts and interactions checked against the schedule, phase times
against the step's own device time, results unchanged by the timing)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def T(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_nb_log_prints_errors_and_launch_choices(monkeypatch, capfd):
    import torch
    import paper_1409_5474_amd as nb
    monkeypatch.setenv("NB_LOG", "2")
    ctx = nb.Context(0, "fp64")
    p = synth.plummer(2048, 7)
    pos, vel, mass = T(p.pos), T(p.vel), T(p.mass)
    act = torch.arange(2048, dtype=torch.int32, device="cuda")
    ctx.forces(pos, vel, mass, act, 1e-4)
    ctx.sync()
    with pytest.raises(nb.NbodyError):
        ctx.forces(pos, vel, mass, act, -1.0)
    ctx.close()
    err = capfd.readouterr().err
    assert "nbody: launch table" in err
    launch = [l for l in err.splitlines() if l.startswith("nbody: forces N=2048 n_active=2048 K=")]
    assert launch, err[-2000:]
    assert any(l.startswith("nbody: error -1: eps2") for l in err.splitlines()), err[-2000:]


def test_nb_log_unset_is_silent(monkeypatch, capfd):
    import torch
    import paper_1409_5474_amd as nb
    monkeypatch.delenv("NB_LOG", raising=False)
    ctx = nb.Context(0, "fp64")
    p = synth.plummer(512, 7)
    act = torch.arange(512, dtype=torch.int32, device="cuda")
    with pytest.raises(nb.NbodyError):
        ctx.forces(T(p.pos), T(p.vel), T(p.mass), act, -1.0)
    ctx.close()
    assert "nbody:" not in capfd.readouterr().err


def test_phase_times_need_a_timed_step():
    import paper_1409_5474_amd as nb
    ctx = nb.Context(0, "fp64")
    with pytest.raises(nb.NbodyError):
        ctx.phase_times()          # timing off
    ctx.set_phase_timing(True)
    with pytest.raises(nb.NbodyError):
        ctx.phase_times()          # no step yet
    ctx.close()


@pytest.mark.parametrize("batch", [False, True], ids=["single", "batch"])
def test_step_records_match_schedule_and_leave_results_unchanged(batch):
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    eta, dt_max, ML = 0.02, 1.0 / 16, 30
    if batch:
        b = synth.cluster_batch(seed=4, n_clusters=6, n_min=128, n_max=1500)
        args = (T(b.pos), T(b.vel), T(b.mass), b.eps2, eta, dt_max, ML)
        kw = dict(offsets=b.offsets)
        sizes = np.diff(b.offsets)
    else:
        p = synth.plummer(4096, 5)
        args = (T(p.pos), T(p.vel), T(p.mass), 1e-4, eta, dt_max, ML)
        kw = {}
    ctx = nb.Context(0, "fp64")
    plain = BlockIntegrator(ctx, *args, **kw)
    timed = BlockIntegrator(ctx, *args, **kw)
    recs = []
    timed.set_metrics(recs.append)
    active_lists = []
    for _ in range(40):
        plain.step()
        timed.step()
        n_act = recs[-1]["n_active"]
        active_lists.append(timed.active[:n_act].cpu().numpy().copy())
    torch.cuda.synchronize()
    assert torch.equal(plain.pos, timed.pos) and torch.equal(plain.vel, timed.vel)
    assert torch.equal(plain.t_tick, timed.t_tick) and torch.equal(plain.level, timed.level)
    assert [r["step"] for r in recs] == list(range(1, 41))
    n = int(timed.n)
    for r, rows in zip(recs, active_lists):
        assert r["kind"] == "step" and r["n_active"] == len(rows) > 0
        if batch:
            sys_of = np.searchsorted(b.offsets, rows, side="right") - 1
            assert r["interactions"] == int(sizes[sys_of].sum())
        else:
            assert r["interactions"] == len(rows) * n
        assert r["ms_schedule"] > 0 and r["ms_forces"] > 0 and r["ms_correct"] > 0
        assert r["ms_schedule"] + r["ms_forces"] + r["ms_correct"] < 50.0
    # the step times are monotone along the run
    ts = [r["t"] for r in recs]
    assert all(a < b for a, b in zip(ts, ts[1:]))
    # graph replays report steps and time; captured steps emit no step records
    n_rec = len(recs)
    timed.run_until(0.125, graph_steps=8)
    new = recs[n_rec:]
    reps = [r for r in new if r["kind"] == "replay"]
    assert reps and all(r["steps"] >= 0 and r["ms"] > 0 for r in reps)
    eager = sum(r["kind"] == "step" and r["n_active"] > 0 for r in new)
    assert sum(r["steps"] for r in reps) + eager == timed.steps - 40
    timed.set_metrics(None)
    with pytest.raises(nb.NbodyError):
        ctx.phase_times()
    ctx.close()


def test_phase_times_cover_the_step():
    # the three phases add up to the device time between events around one step
    import torch
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd.integrator import BlockIntegrator
    p = synth.plummer(16384, 6)
    ctx = nb.Context(0, "mixed")
    bi = BlockIntegrator(ctx, T(p.pos), T(p.vel), T(p.mass), 2.0 ** -16, 0.01, 1.0 / 16, 30)
    ctx.set_phase_timing(True)
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bi.step()
        e1.record()
        torch.cuda.synchronize()
        ms = ctx.phase_times()
        total = e0.elapsed_time(e1)
        assert all(x > 0 for x in ms)
        assert sum(ms) <= total * 1.05 + 0.01
    ctx.close()


def test_nb_tune_cache_names_the_table_a_context_loads(monkeypatch, tmp_path):
    # a table with one distinctive entry: a context created with NB_TUNE_CACHE
    # naming it launches that shape; without the variable, the shipped table
    import paper_1409_5474_amd as nb
    from paper_1409_5474_amd import autotune
    path = tmp_path / "cache.json"
    autotune.save([dict(prec="fp64", n_min=1000, act_min=0, act_max=2 ** 31 - 1, K=1, L=64, items=96)], str(path))
    monkeypatch.setenv("NB_TUNE_CACHE", str(path))
    ctx = nb.Context(0, "fp64")
    assert ctx.tuning_table == str(path)
    assert ctx.get_launch(5000, 3000)[:2] == (1, 64)
    ctx.close()
    monkeypatch.delenv("NB_TUNE_CACHE")
    ctx = nb.Context(0, "fp64")
    assert ctx.tuning_table == autotune.DEFAULT_TABLE
    ctx.close()
