"""Autotuner front end: bucket ranges, table save/load (CPU); a small real
tuning run whose table keeps parity and host/device-count agreement (GPU)."""
import json

import numpy as np
import pytest


def test_bucket_ranges_tile_the_axis():
    from paper_1409_5474_amd import autotune as at
    r = at._midpoints(at.BUCKETS)
    assert r[0][0] == 0 and r[-1][1] == 2 ** 31 - 1
    for (a0, a1), (b0, b1), rep in zip(r[:-1], r[1:], at.BUCKETS):
        assert a1 + 1 == b0 and a0 <= rep <= a1


def test_save_and_load_order(tmp_path):
    from paper_1409_5474_amd import autotune as at
    entries = [dict(prec="mixed", n_min=262144, act_min=0, act_max=10, K=2, L=1, items=0),
               dict(prec="mixed", n_min=65536, act_min=0, act_max=10, K=1, L=4, items=64)]
    p = tmp_path / "t.json"
    at.save(entries, str(p), meta={"device": "test"})
    calls = []

    class FakeCtx:
        def tune_add(self, *a):
            calls.append(a)

    assert at.load(FakeCtx(), str(p)) == 2
    # smaller n_min first, so the larger-N entry overrides it where it applies
    assert [c[1] for c in calls] == [65536, 262144]
    assert json.load(open(p))["meta"]["device"] == "test"


def test_shape_runs_merge_only_within_the_launch_cost():
    # A run of buckets takes a neighbouring run's shape only when that costs
    # each of its buckets at most one launch; merges repeat until none fits,
    # and a bucket's loss never exceeds the launches saved.
    from paper_1409_5474_amd.autotune import _merge_shapes
    A, B, C, D = (1, 256), (1, 64), (1, 16), (2, 1)
    times = [{A: 15, B: 17, C: 20, D: 90}, {A: 18, B: 19, C: 30, D: 80},
             {A: 30, B: 24, C: 25, D: 60}, {A: 60, B: 50, C: 44, D: 50}, {A: 900, B: 400, C: 300, D: 100}]
    fastest = [min(t, key=t.get) for t in times]
    assert fastest == [A, A, B, C, D]
    assert _merge_shapes(fastest, times, 0) == fastest
    got = _merge_shapes(fastest, times, 3)
    assert got == [A, A, C, C, D]          # B -> C costs 1 at bucket 2; nothing else within 3
    saved = len({*fastest}) - len({*got})
    assert all(times[b][got[b]] - times[b][fastest[b]] <= 3 * saved for b in range(5))
    assert _merge_shapes(fastest, times, 10**6) in ([A] * 5, [B] * 5, [C] * 5, [D] * 5)
    # a shape not timed at some bucket of the run (K > 1 below 64 K rows) is never taken there
    t2 = [{A: 10}, {A: 12, D: 12}]
    assert _merge_shapes([A, D], t2, 5) == [A, A]


@pytest.mark.gpu
def test_small_tuning_run_keeps_parity(tmp_path):
    import torch
    import oracle
    import paper_1409_5474_amd as nb
    import synth
    from paper_1409_5474_amd import autotune as at
    ctx = nb.Context(0, "mixed", load_tuning=False)
    entries = at.tune(ctx, 8192, precisions=("mixed",), buckets=[1, 64, 1024, 8192], reps=1, log=lambda s: None)
    assert len(entries) == 4
    path = tmp_path / "tuning.json"
    at.save(entries, str(path))
    ctx2 = nb.Context(0, "mixed", load_tuning=False)
    at.load(ctx2, str(path))
    p = synth.plummer(8192, 2)
    T = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    P, V, M = T(p.pos), T(p.vel), T(p.mass)
    for na in (1, 50, 700, 8192):
        act = np.sort(np.random.default_rng(na).choice(8192, na, replace=False)).astype(np.int32)
        a1, j1, p1 = ctx2.forces(P, V, M, T(act), 2.0 ** -16)
        cnt = torch.tensor([na], dtype=torch.int32, device="cuda")
        full = torch.zeros(8192, dtype=torch.int32, device="cuda")
        full[:na] = T(act)
        a2 = torch.empty((8192, 3), dtype=torch.float64, device="cuda")
        j2, p2 = torch.empty_like(a2), torch.empty(8192, dtype=torch.float64, device="cuda")
        ctx2.forces_devcount(P, V, M, full, cnt, 8192, 2.0 ** -16, a2, j2, p2)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2[:na]) and torch.equal(p1, p2[:na]), na
        ref = oracle.forces_ld(p.pos, p.vel, p.mass, 2.0 ** -16, act[:64])
        err = np.linalg.norm(a1.cpu().numpy()[:64] - ref["acc"], axis=1) / np.linalg.norm(ref["acc"], axis=1)
        assert np.sqrt(np.mean(err ** 2)) < 1e-6, na
