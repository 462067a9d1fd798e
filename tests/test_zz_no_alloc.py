"""nbody_forces_noalloc (the fixed-scratch variant of nbody_forces, for callers
that cannot allocate) against nbody_forces through the C ABI: same launch,
same kernels, so the outputs must be identical bit for bit -- on two calls in
a row, the second smaller than the first, so stale scratch contents from the
first cannot leak into the second.  Where the automatic launch's partial sums
do not fit the fixed scratch, the entry point lowers the j-split: it then
equals nbody_forces forced to that j-split."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

NB_ENOMEM = -2
SCRATCH_BYTES = 256 << 20


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _both(ctx, p, act, eps2):
    n, na = p.mass.shape[0], act.shape[0]
    pos, vel, mass, a = _dev(p.pos), _dev(p.vel), _dev(p.mass), _dev(act)
    ref = ctx.forces(pos, vel, mass, a, eps2)
    out = (torch.full((na, 3), np.nan, dtype=torch.float64, device="cuda:0"),
           torch.full((na, 3), np.nan, dtype=torch.float64, device="cuda:0"),
           torch.full((na,), np.nan, dtype=torch.float64, device="cuda:0"))
    ctx.forces_noalloc(pos, vel, mass, a, eps2, *out)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in out]


def _same(ref, got):
    for r, g in zip(ref, got):
        assert r.tobytes() == g.tobytes()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_nbody_forces_large_then_small(prec):
    import paper_1409_5474_amd as nb
    ctx = nb.Context(0, prec)
    # 1: the benchmark's workload, Plummer N = 262144, all active (scalar
    #    j-path with a j-split, so both the mirror and the partials are used)
    p = synth.plummer(262144, 3)
    eps2 = (1.0 / 256) ** 2
    act = np.arange(262144, dtype=np.int32)
    K, L, S = ctx.get_launch(262144, 262144)
    print(f"noalloc {prec}: N=262144 all active, launch K={K} L={L} S={S}", flush=True)
    ref, got = _both(ctx, p, act, eps2)
    _same(ref, got)
    rows = np.arange(0, 262144, 4099, dtype=np.int32)
    o = oracle.forces_ld(p.pos, p.vel, p.mass, eps2, rows)
    err = np.linalg.norm(got[0][rows] - o["acc"], axis=1) / np.linalg.norm(o["acc"], axis=1)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert (np.sqrt(np.mean(err ** 2)) if prec != "fp64" else err.max()) <= tol
    # 2: a smaller system with a ragged, unsorted active set with duplicates
    q = synth.plummer(5000, 17)
    rng = np.random.default_rng(5)
    act2 = rng.integers(0, 5000, 777).astype(np.int32)
    print(f"noalloc {prec}: N=5000, 777 ragged active", flush=True)
    ref2, got2 = _both(ctx, q, act2, 1e-4)
    _same(ref2, got2)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed_ds"])
def test_noalloc_forced_split_and_rejection(prec):
    import paper_1409_5474_amd as nb
    ctx = nb.Context(0, prec)
    # a forced scalar j-path launch with an 8-way j-split on a ragged size
    ctx.set_launch(2, 0, 8)
    p = synth.plummer(20000, 9)
    act = np.arange(3, 20000, 3, dtype=np.int32)
    print(f"noalloc {prec}: N=20000, forced K=2 L=0 S=8", flush=True)
    ref, got = _both(ctx, p, act, 1e-4)
    _same(ref, got)
    # the same, smaller, after it
    act_s = act[:101]
    ref, got = _both(ctx, p, act_s, 1e-4)
    _same(ref, got)
    # a forced launch whose partials exceed the fixed scratch is refused before
    # any kernel runs: 128 chunks x 56 B x 65536 rows = 470 MB > 256 MiB
    ctx.set_launch(1, 0, 128)
    q = synth.plummer(65536, 2)
    n = 65536
    pos, vel, mass = _dev(q.pos), _dev(q.vel), _dev(q.mass)
    a = _dev(np.arange(n, dtype=np.int32))
    out = [torch.full(s, 7.0, dtype=torch.float64, device="cuda:0") for s in ((n, 3), (n, 3), (n,))]
    with pytest.raises(nb.NbodyError) as ei:
        ctx.forces_noalloc(pos, vel, mass, a, 1e-4, *out)
    assert ei.value.code == NB_ENOMEM and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert all(bool((t == 7.0).all()) for t in out)
    ctx.close()


def test_noalloc_lowers_an_automatic_split_that_does_not_fit():
    import paper_1409_5474_amd as nb
    ctx = nb.Context(0, "mixed", load_tuning=False)
    n = 65536
    # a table entry asking for the most chunks the j-set allows (S = 256):
    # 256 x 56 B x 65536 rows = 940 MB of partials, more than the scratch
    ctx.tune_add("mixed", n, 0, 2 ** 31 - 1, 1, 1, 256 * 256)
    assert ctx.get_launch(n, n) == (1, 1, 256)
    s_fit = (SCRATCH_BYTES - 255) // (56 * n)
    p = synth.plummer(n, 21)
    pos, vel, mass = _dev(p.pos), _dev(p.vel), _dev(p.mass)
    a = _dev(np.arange(n, dtype=np.int32))
    out = [torch.full(sh, np.nan, dtype=torch.float64, device="cuda:0") for sh in ((n, 3), (n, 3), (n,))]
    print(f"noalloc mixed: N=65536 all active, automatic S=256 lowered to {s_fit}", flush=True)
    ctx.forces_noalloc(pos, vel, mass, a, 2.0 ** -16, *out)
    ctx.set_launch(1, 1, s_fit)
    ref = ctx.forces(pos, vel, mass, a, 2.0 ** -16)
    torch.cuda.synchronize()
    _same([t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in out])
    ctx.close()
