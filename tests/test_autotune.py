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


def test_table_path_follows_nb_tune_cache(tmp_path, monkeypatch):
    from paper_1409_5474_amd import autotune as at
    monkeypatch.delenv("NB_TUNE_CACHE", raising=False)
    assert at.table_path() == at.DEFAULT_TABLE
    cache = tmp_path / "cache.json"
    at.save([], str(cache))
    monkeypatch.setenv("NB_TUNE_CACHE", str(cache))
    assert at.table_path() == str(cache)
    # not written yet: the shipped table, with a warning
    monkeypatch.setenv("NB_TUNE_CACHE", str(tmp_path / "later.json"))
    with pytest.warns(UserWarning, match="does not exist yet"):
        assert at.table_path() == at.DEFAULT_TABLE
    monkeypatch.setenv("NB_TUNE_CACHE", "")
    assert at.table_path() == at.DEFAULT_TABLE


def test_jsonl_metrics_sink(tmp_path):
    from paper_1409_5474_amd.integrator import jsonl_sink
    path = tmp_path / "m.jsonl"
    sink = jsonl_sink(str(path))
    sink(dict(kind="step", step=1, n_active=3, interactions=12, ms_forces=0.5))
    sink(dict(kind="replay", steps=8, ms=1.25))
    sink.close()
    lines = [json.loads(l) for l in open(path)]
    assert lines == [dict(kind="step", step=1, n_active=3, interactions=12, ms_forces=0.5),
                     dict(kind="replay", steps=8, ms=1.25)]


def test_shape_runs_merge_only_within_the_launch_cost():
    # A run of buckets that needs a launch of its own takes a neighbouring
    # run's shape only when that costs each of its buckets at most one launch;
    # merges repeat until none fits, and a bucket's loss never exceeds the
    # launches saved.
    from paper_1409_5474_amd.autotune import _merge_shapes, _launch_runs
    A, B, C, D = (1, 256), (2, 0), (4, 1), (2, 1)   # family 1, scalar path, single kernel, family 2
    times = [{A: 15, B: 17, C: 20, D: 90}, {A: 18, B: 19, C: 30, D: 80},
             {A: 30, B: 24, C: 25, D: 60}, {A: 60, B: 50, C: 44, D: 50}, {A: 900, B: 400, C: 300, D: 100}]
    fastest = [min(t, key=t.get) for t in times]
    assert fastest == [A, A, B, C, D]
    assert _merge_shapes(fastest, times, 0) == fastest
    got = _merge_shapes(fastest, times, 3)
    assert got == [A, A, C, C, D]          # B -> C costs 1 at bucket 2; nothing else within 3
    saved = len(_launch_runs(fastest)) - len(_launch_runs(got))
    assert saved == 1
    assert all(times[b][got[b]] - times[b][fastest[b]] <= 3 * saved for b in range(5))
    assert len(_launch_runs(_merge_shapes(fastest, times, 10**6))) == 1
    # a shape not timed at some bucket of the run (K > 1 below 64 K rows) is never taken there
    t2 = [{A: 10}, {A: 12, (2, 0): 12}]
    assert _merge_shapes([A, (2, 0)], t2, 5) == [A, A]


def test_one_bucket_changes_shape_when_that_alone_saves_a_launch():
    # K = 4, L = 4 (family 4) between K = 1 shapes and the K = 2 shapes of
    # family 2 keeps two launches per step; the bucket takes its best family-2
    # shape when that costs at most one launch, and keeps its own otherwise.
    from paper_1409_5474_amd.autotune import _merge_shapes, _launch_runs
    K1a, K1b, K44, K24, K21 = (1, 64), (1, 4), (4, 4), (2, 4), (2, 1)
    fastest = [K1a, K1b, K44, K24, K21]
    assert len(_launch_runs(fastest)) == 2
    def times_with(pen):
        return [{K1a: 10, K1b: 12}, {K1a: 20, K1b: 15}, {K44: 50, K1b: 50 + pen, K24: 50 + 2 * pen, K1a: 90},
                {K24: 100, K21: 104}, {K21: 400, K24: 420}]
    got = _merge_shapes(fastest, times_with(1.5), 3)
    assert got == [K1a, K1b, K1b, K24, K21] and len(_launch_runs(got)) == 1
    assert _merge_shapes(fastest, times_with(4), 3) == fastest


def test_shapes_one_family_holds_share_a_launch():
    # LDS shapes of one kernel family run in one device-count launch, so the
    # merge keeps each bucket's fastest shape there
    from paper_1409_5474_amd.autotune import _merge_shapes, _launch_runs, _family
    ch = [(1, 64), (1, 4), (2, 4), (2, 1), (2, 1)]
    times = [{sh: 1.0 + 0.001 * k for k, sh in enumerate(ch)} for _ in ch]
    assert len(_launch_runs(ch)) == 1
    assert _merge_shapes(ch, times, 10**6) == ch
    # other tile lengths / workgroup sizes, the scalar path and (4, 1) are single kernels
    assert [_family(s) for s in [(1, 1, 128, 128), (2, 0), (4, 1), (4, 4), (1, 256)]] == [0, 0, 0, 4, 1]
    assert len(_launch_runs([(1, 4), (4, 4), (2, 1)])) == 2   # families 2 and 4 hold different K


def test_shipped_table_covers_every_tuned_workload():
    # The table loaded by default: every precision has single-system entries
    # for N = 65536, 262144 and 1441803 whose active-count ranges tile
    # [0, 2^31), and batched entries (both kinds) over every key; the force
    # kernels' source hash it was measured on is recorded.
    from paper_1409_5474_amd import autotune as at
    doc = json.load(open(at.DEFAULT_TABLE))
    assert len(doc["meta"]["forces_hip_sha256"]) == 64
    entries = doc["entries"]
    for prec in ("fp64", "mixed", "mixed_ds"):
        for n in (65536, 262144, 1441803):
            es = sorted((e for e in entries if e.get("kind", 0) == 0 and e["prec"] == prec and e["n_min"] == n),
                        key=lambda e: e["act_min"])
            assert es and es[0]["act_min"] == 0 and es[-1]["act_max"] == 2 ** 31 - 1, (prec, n)
            assert all(a["act_max"] + 1 == b["act_min"] for a, b in zip(es, es[1:])), (prec, n)
            assert all("T" in e and "WG" in e for e in es)
        for kind in (1, 2):
            es = sorted((e for e in entries if e.get("kind", 0) == kind and e["prec"] == prec),
                        key=lambda e: e["key_min"])
            assert es and es[0]["key_min"] <= 1 and es[-1]["key_max"] == 2 ** 31 - 1, (prec, kind)
            assert all(a["key_max"] + 1 == b["key_min"] for a, b in zip(es, es[1:])), (prec, kind)
        # the batched workloads' systems (128 to 16384 bodies) each fall in a tuned kind-1 range
        for size in (128, 1000, 3344, 16384):
            assert any(e["key_min"] <= size <= e["key_max"] for e in entries
                       if e.get("kind", 0) == 1 and e["prec"] == prec)


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
