"""GPU parity of the force kernels against the CPU oracle (extended
precision), through the C ABI.  Gates:
  FP64 : per particle |da_i| <= 1e-12 |a_i| + 64 eps64 A_i (A_i = sum_j |a_ij|)
         and normwise ||da||/||a|| <= 1e-12, for acc, jerk and pot
  mixed: RMS_i |da_i|/|a_i| <= 1e-6 for acc; jerk <= 1e-5; pot <= 1e-6
"""
import numpy as np
import pytest

import oracle
import synth
from errors import all_errs, check_fp64, check_mixed

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -53
PRECS = ["fp64", "mixed", "mixed_ds"]


@pytest.fixture(scope="module")
def nb():
    import paper_1409_5474_amd as nbm
    return nbm


@pytest.fixture(scope="module")
def ctx(nb):
    c = nb.Context(0, "fp64")
    yield c
    c.close()


def _dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def run_gpu(ctx, prec, p, eps2, active, launch=None):
    import torch
    ctx.set_precision(prec)
    if launch:
        ctx.set_launch(*launch)
    else:
        ctx.set_launch(0)
    acc, jerk, pot = ctx.forces(_dev(p.pos), _dev(p.vel), _dev(p.mass), _dev(active.astype(np.int32)), eps2)
    torch.cuda.synchronize()
    ctx.set_launch(0)
    return acc.cpu().numpy(), jerk.cpu().numpy(), pot.cpu().numpy()


def _case(n, seed):
    return synth.plummer(n, seed)


@pytest.mark.parametrize("prec", PRECS)
def test_small_plummer_all_active(ctx, prec):
    # Plummer N = 1024, eps = 0.01, every particle active.
    p = _case(1024, 1)
    eps2 = synth.plummer_eps2_c1()
    act = np.arange(1024, dtype=np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)
    res = run_gpu(ctx, prec, p, eps2, act)
    if prec == "fp64":
        check_fp64(res, ref)
    else:
        check_mixed(res, ref)


# (K, L, S); L = 0 is the scalar j-path
LAUNCHES = [(1, 1, 1), (2, 1, 1), (4, 1, 1), (1, 1, 3), (2, 1, 5), (1, 2, 1), (1, 4, 2), (2, 8, 3), (4, 16, 1),
            (1, 32, 2), (2, 64, 4), (1, 128, 1), (1, 256, 7), (4, 4, 4), (2, 32, 2), (1, 0, 1), (2, 0, 3), (3, 0, 2), (1, -1, 1), (2, -1, 3), (3, -1, 2),
            (4, 0, 1), (2, 0, 1),
            # (K, L, S, T, WG): other j-tile lengths and workgroup sizes
            (1, 1, 2, 128, 128), (2, 4, 3, 128, 256), (1, 16, 5, 64, 64), (2, 1, 1, 64, 64), (1, 4, 7, 128, 256),
            (2, 1, 9, 128, 128), (1, 0, 3, 0, 128), (2, 0, 2, 0, 128)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("launch", LAUNCHES)
def test_every_launch_shape_ragged(ctx, prec, launch):
    # N not a multiple of the tile, an active set not a multiple of the i-block.
    n = 3001
    p = _case(n, 7)
    eps2 = 1e-3
    rng = np.random.default_rng(3)
    act = np.sort(rng.choice(n, 777, replace=False)).astype(np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)
    res = run_gpu(ctx, prec, p, eps2, act, launch)
    if prec == "fp64":
        check_fp64(res, ref)
    else:
        check_mixed(res, ref)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_act", [1, 7, 63, 64, 65, 1000, 4096])
def test_active_set_sizes(ctx, prec, n_act):
    n = 4096
    p = _case(n, 9)
    eps2 = 2.0 ** -16
    rng = np.random.default_rng(n_act)
    act = np.sort(rng.choice(n, n_act, replace=False)).astype(np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)
    res = run_gpu(ctx, prec, p, eps2, act)
    if prec == "fp64":
        check_fp64(res, ref)
    else:
        check_mixed(res, ref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_duplicates_and_unsorted(ctx, prec):
    p = _case(500, 4)
    act = np.array([499, 3, 3, 250, 0, 3, 499], dtype=np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, 1e-3, act)
    res = run_gpu(ctx, prec, p, 1e-3, act)
    (check_fp64 if prec == "fp64" else check_mixed)(res, ref)
    # duplicated rows are bitwise equal
    for arr in res:
        assert np.array_equal(arr[1], arr[2]) and np.array_equal(arr[1], arr[5])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiny_systems(ctx, prec):
    # N = 1: no other particle -> zeros; N = 2: the two-body closed form.
    import types
    one = types.SimpleNamespace(pos=np.zeros((1, 3)), vel=np.zeros((1, 3)), mass=np.ones(1))
    res = run_gpu(ctx, prec, one, 0.01, np.array([0], np.int32))
    for arr in res:
        assert np.all(arr == 0.0)
    two = types.SimpleNamespace(pos=np.array([[0.0, 0, 0], [1.5, 0, 0]]), vel=np.zeros((2, 3)),
                                mass=np.array([0.3, 0.7]))
    res = run_gpu(ctx, prec, two, 0.04, np.array([0, 1], np.int32))
    tol = 1e-15 if prec == "fp64" else 1e-6
    s32 = (1.5 ** 2 + 0.04) ** 1.5
    assert res[0][0, 0] == pytest.approx(0.7 * 1.5 / s32, rel=tol)
    assert res[0][1, 0] == pytest.approx(-0.3 * 1.5 / s32, rel=tol)
    assert res[2][0] == pytest.approx(-0.7 / np.sqrt(1.5 ** 2 + 0.04), rel=tol)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L", [1, 0])
def test_zero_softening_masks_coincident_pairs(ctx, prec, L):
    # eps2 = 0: the self pair and a coincident twin contribute nothing.
    p = _case(300, 5)
    pos = p.pos.copy()
    pos[10] = pos[20]
    import types
    q = types.SimpleNamespace(pos=pos, vel=p.vel, mass=p.mass)
    act = np.arange(300, dtype=np.int32)
    ref = oracle.forces_ld(pos, p.vel, p.mass, 0.0, act)
    assert ref["skipped"] == 2
    res = run_gpu(ctx, prec, q, 0.0, act, (1, L, 2))
    for arr in res:
        assert np.all(np.isfinite(arr))
    if prec == "fp64":
        check_fp64(res, ref)
        return
    # Unsoftened, the closest pairs dominate each sum and partly cancel, so a
    # row's float rounding is bounded by the sum of its terms' magnitudes, not
    # by its result: |d_i| <= 64 u sum_j |term_ij| with u = 2^-24 (float runs
    # of up to 32 pairs, plus the rounding of r and of the pair terms).
    u = 2.0 ** -24
    for name, got in zip(("acc", "jerk", "pot"), res):
        err = np.abs(got - ref[name]) if got.ndim == 1 else np.linalg.norm(got - ref[name], axis=1)
        bound = 64 * u * ref["abs_" + name]    # the oracle's per-row sums of |term_ij|
        assert (err <= bound).all(), (name, (err / bound).max())
    # rows whose sums are well conditioned meet the standard gate
    a = np.linalg.norm(ref["acc"], axis=1)
    ok = ref["abs_acc"] < 20 * a
    rel = np.linalg.norm(res[0][ok] - ref["acc"][ok], axis=1) / a[ok]
    assert ok.sum() > 150 and np.sqrt(np.mean(rel ** 2)) <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n,S", [(66000, 3), (66000, 7), (66000, 13), (66000, 61), (66000, 256), (160000, 600)])
def test_split_sum_over_many_blocks(ctx, prec, n, S):
    # A few rows against up to 600 j-blocks: the partial sums of one output
    # are added by 1 to 64 lanes (at most four blocks each up to S = 256,
    # more beyond) and folded.
    p = _case(n, 31)
    act = np.array([0, 17, 17, 40000, n - 1], dtype=np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, 2.0 ** -16, act)
    res = run_gpu(ctx, prec, p, 2.0 ** -16, act, (1, 64, S))
    (check_fp64 if prec == "fp64" else check_mixed)(res, ref)
    for arr in res:
        assert np.array_equal(arr[1], arr[2])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("launch", [(1, 4, 3), (2, 0, 2)])
def test_bitwise_deterministic(ctx, prec, launch):
    p = _case(5000, 6)
    act = np.arange(0, 5000, 3, dtype=np.int32)
    r1 = run_gpu(ctx, prec, p, 1e-3, act, launch)
    r2 = run_gpu(ctx, prec, p, 1e-3, act, launch)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_sampled(ctx, prec):
    # Plummer N = 262144, eps = 1/256, all active in the launch the benchmark
    # uses; 512 sampled rows checked against the oracle one by one.
    n = 262144
    p = _case(n, 3)
    eps2 = 2.0 ** -16
    act = np.arange(n, dtype=np.int32)
    res = run_gpu(ctx, prec, p, eps2, act)
    rows = np.sort(np.random.default_rng(11).choice(n, 512, replace=False)).astype(np.int32)
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, rows)
    sub = tuple(a[rows] for a in res)
    if prec == "fp64":
        check_fp64(sub, ref)
    else:
        check_mixed(sub, ref)
    # Newton's third law over the whole system (exact in exact arithmetic)
    a = res[0]
    fa = np.linalg.norm((p.mass[:, None] * a).sum(0))
    scale = (p.mass * np.linalg.norm(a, axis=1)).sum()
    assert fa <= (1e-13 if prec == "fp64" else 1e-6) * scale


def test_workspace_cap_reports_enomem_without_writing(ctx):
    # A j-split needs a workspace; a cap below its size must fail with
    # NB_ENOMEM (-2) before anything is launched, and leave outputs untouched.
    import os
    import subprocess
    import sys
    code = r'''
import sys, numpy as np, torch
sys.path.insert(0, %r)
import paper_1409_5474_amd as nb, synth
p = synth.plummer(4096, 3)
ctx = nb.Context(0, "fp64", load_tuning=False)
ctx.set_launch(1, 64, 32)
t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
acc = torch.full((16, 3), 7.0, dtype=torch.float64, device="cuda")
jerk = torch.full((16, 3), 7.0, dtype=torch.float64, device="cuda")
pot = torch.full((16,), 7.0, dtype=torch.float64, device="cuda")
try:
    ctx.forces(t(p.pos), t(p.vel), t(p.mass), torch.arange(16, dtype=torch.int32, device="cuda"), 1e-4, acc, jerk, pot)
    print("NO-ERROR")
except nb.NbodyError as e:
    torch.cuda.synchronize()
    print("CODE", e.code, bool((acc == 7.0).all() and (pot == 7.0).all()))
''' % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, NB_MAX_WORKSPACE_BYTES="1024")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert "CODE -2 True" in r.stdout, (r.stdout, r.stderr[-2000:])


def test_workspace_growth_stays_within_the_cap(ctx):
    # A request just under the cap succeeds and the workspace it grows stays
    # within the cap (growth headroom is clamped to it).
    import os
    import subprocess
    import sys
    code = r'''
import sys, numpy as np, torch
sys.path.insert(0, %r)
import paper_1409_5474_amd as nb, synth
p = synth.plummer(4096, 3)
ctx = nb.Context(0, "fp64", load_tuning=False)
ctx.set_launch(1, 64, 32)
t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
acc, jerk, pot = ctx.forces(t(p.pos), t(p.vel), t(p.mass), torch.arange(16, dtype=torch.int32, device="cuda"), 1e-4)
torch.cuda.synchronize()
print("BYTES", ctx.workspace_bytes(), bool(torch.isfinite(acc).all()))
''' % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    need = 16 * 7 * 16 * 8      # S x 7 x n_active doubles (S = 32 is capped at N / 256 = 16 chunks)
    env = dict(os.environ, NB_MAX_WORKSPACE_BYTES=str(need + 100))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert "BYTES" in r.stdout, (r.stdout, r.stderr[-2000:])
    got = r.stdout.split("BYTES")[1].split()
    assert need <= int(got[0]) <= need + 100 and got[1] == "True", r.stdout


# ---- i-set entries outside their valid range -------------------------------
# Every kernel that reads active_idx tests each entry first: a bad entry gets
# no output row and nothing is read through it; the context's device error
# word records it, and the next nb_sync reports NB_EINVAL once.

def _with_bad(valid, n, at, bad):
    a = list(valid)
    for pos_, b in zip(at, bad):
        a.insert(pos_, b)
    return np.array(a, dtype=np.int32)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(2, 0, 4), (1, 16, 4), (1, 1, 1)])
def test_out_of_range_entries_are_skipped_and_reported(nb, prec, shape):
    import torch
    c = nb.Context(0, prec, load_tuning=False)
    n = 5000
    p = synth.plummer(n, 31)
    P, V, M = _dev(p.pos), _dev(p.vel), _dev(p.mass)
    valid = np.arange(0, n, 7, dtype=np.int32)
    bad_at, bad = [0, 100, 300], [-1, n, 2 ** 31 - 1]
    act = _with_bad(valid, n, bad_at, bad)
    isbad = np.isin(np.arange(act.size), bad_at)
    c.set_launch(*shape)
    print(f"range check {prec} K,L,S={shape}: {act.size} entries, {len(bad)} bad", flush=True)
    out = [torch.full(s, 7.0, dtype=torch.float64, device="cuda") for s in ((act.size, 3), (act.size, 3), (act.size,))]
    c.forces(P, V, M, _dev(act), 1e-3, *out)
    with pytest.raises(nb.NbodyError) as ei:
        c.sync()
    assert ei.value.code == -1 and "active_idx" in str(ei.value)
    c.sync()                                   # reported once, then clear
    ref = c.forces(P, V, M, _dev(valid), 1e-3)
    torch.cuda.synchronize()
    for o, r in zip(out, ref):
        o = o.cpu().numpy(); r = r.cpu().numpy()
        assert np.all(o[isbad] == 7.0)
        assert o[~isbad].tobytes() == r.tobytes()
    c.close()


def test_out_of_range_entries_in_the_other_entry_points(nb):
    import torch
    c = nb.Context(0, "fp64")
    n = 3000
    p = synth.plummer(n, 32)
    P, V, M = _dev(p.pos), _dev(p.vel), _dev(p.mass)
    # separate i-set: N_i = 40 rows, one entry 40
    pi = synth.plummer(40, 33)
    act = np.array([0, 39, 40, 5], np.int32)
    out = [torch.full(s, 7.0, dtype=torch.float64, device="cuda") for s in ((4, 3), (4, 3), (4,))]
    c.forces_ij(P, V, M, _dev(pi.pos), _dev(pi.vel), _dev(act), 1e-3, *out)
    with pytest.raises(nb.NbodyError):
        c.sync()
    assert bool((out[0][2] == 7.0).all()) and bool((out[0][3] != 7.0).all())
    # batch: system 1 owns rows [1000, 3000); an entry of system 0 in its list
    off = np.array([0, 1000, n], np.int64)
    act_b = np.array([3, 999, 1000, 5, 2999], np.int32)       # 5 lies in system 0, listed under system 1
    aoff = np.array([0, 2, 5], np.int64)
    out = [torch.full(s, 7.0, dtype=torch.float64, device="cuda") for s in ((5, 3), (5, 3), (5,))]
    c.forces_batch(off, [1e-3, 1e-3], P, V, M, _dev(act_b), aoff, *out)
    with pytest.raises(nb.NbodyError):
        c.sync()
    assert bool((out[2][3] == 7.0).all()) and bool((out[2][[0, 1, 2, 4]] != 7.0).all())
    # snap kernel
    act6 = np.array([1, n, 2], np.int32)
    a6 = [torch.full(s, 7.0, dtype=torch.float64, device="cuda") for s in ((3, 3), (3, 3), (3, 3), (3,))]
    c.forces6(P, V, torch.zeros_like(P), M, _dev(act6), 1e-3, *a6)
    with pytest.raises(nb.NbodyError):
        c.sync()
    assert bool((a6[0][1] == 7.0).all()) and bool((a6[0][0] != 7.0).all())
    # corrector: an entry N touches nothing; the valid rows are corrected
    pos, vel = _dev(p.pos), _dev(p.vel)
    acc = torch.zeros_like(pos); jerk = torch.zeros_like(pos)
    tt = torch.zeros(n, dtype=torch.int64, device="cuda"); lv = torch.zeros(n, dtype=torch.int32, device="cuda")
    actc = np.array([7, n, 9], np.int32)
    a1 = torch.ones((3, 3), dtype=torch.float64, device="cuda"); j1 = torch.zeros_like(a1)
    before = pos.clone()
    c.correct(_dev(actc), pos.clone(), vel.clone(), a1, j1, pos, vel, acc, jerk, tt, lv, 0.01, 1.0 / 16, 20)
    with pytest.raises(nb.NbodyError):
        c.sync()
    changed = (pos != before).any(1).cpu().numpy()
    assert changed[7] and changed[9] and changed.sum() == 2
    c.sync()
    c.close()


def test_tuned_tile_and_workgroup_shapes_host_and_device_count(ctx):
    # Table entries with other (T, WG) drive both launch kinds: every count
    # gets the same bits from a host-count and a device-count launch, and
    # the oracle's values.
    import torch
    n = 5000
    p = _case(n, 13)
    eps2 = 1e-3
    P, V, M = _dev(p.pos), _dev(p.vel), _dev(p.mass)
    for prec in PRECS:
        c = __import__("paper_1409_5474_amd").Context(0, prec, load_tuning=False)
        c.tune_add(prec, 1, 0, 40, 1, 16, 0, 64, 64)
        c.tune_add(prec, 1, 41, 900, 2, 4, 0, 128, 256)
        c.tune_add(prec, 1, 901, 2 ** 31 - 1, 2, 1, 0, 128, 128)
        assert c.get_shape(n, 20)[3:] == (64, 64) and c.get_shape(n, 3000)[3:] == (128, 128)
        for na in (7, 300, 3000):
            act = np.sort(np.random.default_rng(na).choice(n, na, replace=False)).astype(np.int32)
            a1, j1, p1 = c.forces(P, V, M, _dev(act), eps2)
            cnt = torch.tensor([na], dtype=torch.int32, device="cuda")
            a2 = torch.empty((n, 3), dtype=torch.float64, device="cuda"); j2 = torch.empty_like(a2)
            p2 = torch.empty(n, dtype=torch.float64, device="cuda")
            act_full = torch.zeros(n, dtype=torch.int32, device="cuda"); act_full[:na] = _dev(act)
            c.forces_devcount(P, V, M, act_full, cnt, n, eps2, a2, j2, p2)
            torch.cuda.synchronize()
            assert torch.equal(a1, a2[:na]) and torch.equal(j1, j2[:na]) and torch.equal(p1, p2[:na]), (prec, na)
            ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)
            res = (a1.cpu().numpy(), j1.cpu().numpy(), p1.cpu().numpy())
            if prec == "fp64":
                check_fp64(res, ref)
            else:
                check_mixed(res, ref)
        c.sync()
        c.close()


def test_unbuilt_tile_shapes_are_rejected(ctx):
    import paper_1409_5474_amd as nb
    for shape in ((1, 64, 1, 128, 128), (4, 1, 1, 128, 256), (1, 4, 1, 96, 128), (3, 0, 1, 0, 128)):
        with pytest.raises(nb.NbodyError):
            ctx.set_launch(*shape)
    ctx.set_launch(0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("launch", [(1, 1, 5), (1, 16, 40), (2, 4, 9), (1, 64, 64), (2, 1, 3)])
def test_atomic_split_sum_equals_the_fixed_order_sum(nb, prec, launch):
    # The paper's two ways of adding the partial forces of a j-split agree:
    # every subset's partial sums are the same numbers either way, and only
    # the order of the S additions differs (atomics: run-dependent).
    import torch
    n = 20000
    p = _case(n, 21)
    eps2 = 1e-3
    act = np.sort(np.random.default_rng(4).choice(n, 3000, replace=False)).astype(np.int32)
    c = nb.Context(0, prec, load_tuning=False)
    c.set_launch(*launch)
    P, V, M, A = _dev(p.pos), _dev(p.vel), _dev(p.mass), _dev(act)
    fixed = [x.cpu().numpy() for x in c.forces(P, V, M, A, eps2)]
    c.set_split_sum(1)
    atomic = [x.cpu().numpy() for x in c.forces(P, V, M, A, eps2)]
    torch.cuda.synchronize()
    for f, a in zip(fixed, atomic):
        if f.ndim == 2:
            scale = np.linalg.norm(f, axis=1)
            diff = np.linalg.norm(a - f, axis=1)
        else:
            scale, diff = np.abs(f), np.abs(a - f)
        assert (diff <= 1e-12 * scale + 1e-300).all(), (diff / scale).max()
    ref = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, act)
    (check_fp64 if prec == "fp64" else check_mixed)(tuple(atomic), ref)
    # shapes the atomic form does not run, and eps2 = 0, are refused
    c.set_launch(2, 0, 4)
    with pytest.raises(nb.NbodyError):
        c.forces(P, V, M, A, eps2)
    c.set_launch(*launch)
    with pytest.raises(nb.NbodyError):
        c.forces(P, V, M, A, 0.0)
    c.set_split_sum(0)
    c.sync()
    c.close()
