"""Autotuner for the force kernel's launch shape.

For each precision and each active-set bucket it times every built
(K, L) shape over a range of j-subset counts S with ``nb_time_forces`` (HIP
events on the context stream); a second stage times the two fastest shapes
with every other j-tile length T and workgroup size WG built for them.  The
winner is stored as a table entry (K, L, T, WG, work-item target = S x
i-blocks) covering the active counts between the geometric midpoints of
neighbouring buckets; the library derives S from that target with the
paper's saturation rule, identically for host-count and device-count
launches.  ``tune_batch_forces`` and ``tune_batch_steps`` tune the batched
kernel (the latter inside graph-replayed block steps).

A block step launches one kernel per distinct shape of the table (each
returns at once unless the device-held count falls in its range), so every
shape run costs about one empty launch in every step.  After the sweep, a
run of buckets takes a neighbouring run's shape when that costs it at most
``launch_ms`` at each of its buckets: a step's count falls in one bucket, so
the switch loses at most that much in a step and always saves one launch.
A single bucket likewise takes another shape when that alone saves a launch
(e.g. a shape of one kernel family where its fastest keeps two families
apart).

    python -m paper_1409_5474_amd.autotune --n 65536 262144 --out tuning.json

``load(ctx, path)`` installs a saved table into a context.
"""
import argparse
import json
import math
import os
import sys
import time
import warnings

import numpy as np
import torch

# (K, L); L = 0 is the scalar j-path (i-parallel, j-records through the scalar cache)
SHAPES = [(1, 1), (1, 4), (1, 16), (1, 64), (1, 256), (2, 1), (2, 4), (2, 16), (4, 1), (4, 4), (1, 0), (2, 0), (3, 0), (4, 0)]
BUCKETS = [1, 8, 64, 256, 1024, 4096, 16384, 65536, 262144]
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
TILE, WG = 256, 256
# Second stage: the j-tile length T and workgroup size WG the library builds
# besides (256, 256), per (K, L) (see nb_set_launch).
TILE_WG = {(1, 1): [(128, 256), (128, 128), (64, 64)], (1, 4): [(128, 256), (128, 128), (64, 64)],
           (1, 16): [(128, 256), (128, 128), (64, 64)], (2, 1): [(128, 256), (128, 128), (64, 64)],
           (2, 4): [(128, 256), (128, 128), (64, 64)], (1, 0): [(256, 128)], (2, 0): [(256, 128)]}


# j-split counts tried: every S up to 8, then steps of about a quarter.  The
# time is not monotone in S (items are handed out from a queue, and how the
# last items fall across the compute units matters), so powers of two alone
# miss good values.
_S_STEPS = [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 128, 160, 192, 256]


def _s_candidates(n, n_act, K, L, num_cus, tile=TILE, wg=WG):
    ib = (wg // max(L, 1)) * K
    n_iblk = -(-n_act // ib)
    max_s = -(-n // tile)
    out = {0}
    for s in _S_STEPS:
        if s > max_s or n_iblk * s > 32 * num_cus:
            break
        out.add(s)
    return sorted(out), n_iblk


def _full(sh):
    """(K, L) or (K, L, T, WG) -> (K, L, T, WG)."""
    return tuple(sh) if len(sh) == 4 else (sh[0], sh[1], TILE, WG)


def _shape_str(sh):
    K, L, tl, wg = _full(sh)
    return f"K={K} L={L} T={tl} WG={wg}"


def _midpoints(buckets):
    lo = [0]
    for a, b in zip(buckets[:-1], buckets[1:]):
        lo.append(int(math.floor(math.sqrt(a * b))) + 1)
    hi = [x - 1 for x in lo[1:]] + [2 ** 31 - 1]
    return list(zip(lo, hi))


# cost of one empty force launch in a graph-replayed block step (measured
# 3.5-5 us per launch on MI355X; the smaller figure keeps the merge safe)
LAUNCH_MS = 0.003


def _family(sh):
    """The library's family_of: the LDS kernel family holding a shape (0: none)."""
    K, L, tl, wg = _full(sh)
    if tl != TILE or wg != WG or L < 1:
        return 0
    if K == 1 and L in (1, 4, 16, 64, 256):
        return 1
    if K == 2 and L in (1, 4, 16):
        return 2
    if K == 4 and L == 4:
        return 4
    return 0


def _cover(a, b):
    """The library's family_cover."""
    if not a or not b:
        return 0
    if a == b or b == 1:
        return a
    if a == 1:
        return b
    return 0


def _launch_runs(choice):
    """Runs of buckets that share one device-count launch: the same shape, or
    shapes one kernel family holds.  Returns [(family or None, [buckets])]."""
    runs = []
    for b, sh in enumerate(choice):
        if runs:
            fam, bs = runs[-1]
            if choice[bs[-1]] == sh and fam is None:
                bs.append(b)
                continue
            joint = _cover(fam if fam else _family(choice[bs[-1]]), _family(sh))
            if joint:
                runs[-1] = (joint, bs + [b])
                continue
        runs.append((None, [b]))
    return runs


def _merge_buckets(choice, times, launch_ms):
    """One bucket at a time: a bucket takes another of its timed shapes when
    that lowers the number of launch runs at a cost of at most launch_ms
    (the cheapest such change first, repeated until none fits) -- e.g. the
    one bucket whose shape keeps two kernel families from sharing a launch."""
    choice = list(choice)
    while True:
        n_runs = len(_launch_runs(choice))
        best = None
        for b, t in enumerate(times):
            for sh, ms in t.items():
                pen = ms - t[choice[b]]
                if sh == choice[b] or pen > launch_ms or (best is not None and pen >= best[0]):
                    continue
                if len(_launch_runs(choice[:b] + [sh] + choice[b + 1:])) < n_runs:
                    best = (pen, b, sh)
        if best is None:
            return choice
        choice[best[1]] = best[2]


def _merge_shapes(choice, times, launch_ms):
    """choice[b]: the shape of bucket b; times[b]: {shape: best ms}.  Returns
    the choice after merging launch runs into neighbours (see module doc): a
    run whose buckets all take the shape of the neighbouring run's nearest
    bucket at a cost of at most launch_ms each saves one launch per step;
    then single buckets as in _merge_buckets, and again until neither
    changes anything.  Every change saves a launch and costs a bucket at
    most launch_ms, so no bucket loses more than the launches saved."""
    while True:
        merged = _merge_runs(choice, times, launch_ms)
        merged = _merge_buckets(merged, times, launch_ms)
        if merged == list(choice):
            return merged
        choice = merged


def _merge_runs(choice, times, launch_ms):
    choice = list(choice)
    while True:
        runs = _launch_runs(choice)
        best = None
        for r, (_, bs) in enumerate(runs):
            for q in (r - 1, r + 1):
                if not 0 <= q < len(runs):
                    continue
                other = choice[runs[q][1][-1] if q < r else runs[q][1][0]]
                if not all(other in times[b] for b in bs):
                    continue
                pen = max(times[b][other] - times[b][choice[b]] for b in bs)
                if pen <= launch_ms and (best is None or pen < best[0]):
                    best = (pen, bs, other)
        if best is None:
            return choice
        for b in best[1]:
            choice[b] = best[2]


def tune(ctx, n, precisions=("fp64", "mixed", "mixed_ds"), buckets=BUCKETS, seed=2, reps=3, log=print,
         launch_ms=LAUNCH_MS):
    import synth
    dev = ctx.device
    p = synth.plummer(n, seed)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    P, V, M = t(p.pos), t(p.vel), t(p.mass)
    eps2 = 2.0 ** -16
    num_cus = torch.cuda.get_device_properties(dev).multi_processor_count
    bks = [b for b in buckets if b <= n]
    ranges = _midpoints(bks)
    entries = []
    for prec in precisions:
        ctx.set_precision(prec)
        times, best_of = [], []
        for b in bks:
            act = torch.from_numpy(np.linspace(0, n - 1, b).astype(np.int32)).to(dev)
            acc = torch.empty((b, 3), dtype=torch.float64, device=dev)
            jerk = torch.empty_like(acc)
            pot = torch.empty(b, dtype=torch.float64, device=dev)
            per_shape = {}
            for K, L in SHAPES:
                if K > 1 and b < 64 * K:
                    continue
                svals, n_iblk = _s_candidates(n, b, K, L, num_cus)
                for S in svals:
                    r = reps if b * n < 2 ** 32 else max(1, reps - 1)
                    ms = ctx.time_forces(K, L, S, P, V, M, act, eps2, acc, jerk, pot, reps=r)
                    if (K, L) not in per_shape or ms < per_shape[(K, L)][0]:
                        per_shape[(K, L)] = (ms, S, n_iblk)
            # second stage: the two fastest shapes with every other (T, WG)
            # built for them, at j-splits around their best (scaled to keep
            # the work-item count)
            base = sorted(per_shape.items(), key=lambda kv: kv[1][0])[:2]
            for (K, L), (ms0, S0, _) in base:
                for tl, wg in TILE_WG.get((K, L), []):
                    svals, n_iblk = _s_candidates(n, b, K, L, num_cus, tl, wg)
                    ib0 = (WG // max(L, 1)) * K
                    ib = (wg // max(L, 1)) * K
                    centre = max(1, round(S0 * (-(-b // ib0)) / max(1, -(-b // ib)))) if S0 else 0
                    near = sorted({0} | {v for v in svals if centre and centre / 2 <= v <= centre * 2})
                    for S in near:
                        ms = ctx.time_forces(K, L, S, P, V, M, act, eps2, acc, jerk, pot, reps=reps, T=tl, WG=wg)
                        key = (K, L, tl, wg)
                        if key not in per_shape or ms < per_shape[key][0]:
                            per_shape[key] = (ms, S, n_iblk)
            times.append({sh: v[0] for sh, v in per_shape.items()})
            best_of.append(per_shape)
            sh, v = min(per_shape.items(), key=lambda kv: kv[1][0])
            log(f"# {prec} N={n} n_active={b}: fastest {_shape_str(sh)} S={v[1]} {v[0]:.5f} ms")
        fastest = [min(t, key=t.get) for t in times]
        choice = _merge_shapes(fastest, times, launch_ms)
        for i, (b, (lo, hi)) in enumerate(zip(bks, ranges)):
            K, L, tl, wg = _full(choice[i])
            ms, S, n_iblk = best_of[i][choice[i]]
            items = S * n_iblk if S else 0
            e = dict(prec=prec, n_min=n, act_min=lo, act_max=hi, K=K, L=L, T=tl, WG=wg, items=items,
                     ms=round(ms, 5), rep_n_active=b, gint=round(b * n / ms / 1e6, 2))
            if choice[i] != fastest[i]:
                fK, fL, fT, fW = _full(fastest[i])
                e["fastest"] = dict(K=fK, L=fL, T=fT, WG=fW, ms=round(times[i][fastest[i]], 5))
            entries.append(e)
            log(json.dumps(e))
    return entries


# Shapes of the batched force kernel (L = 0: scalar j-path)
BATCH_SHAPES = [(1, 1), (1, 4), (1, 16), (1, 64), (2, 1), (2, 4), (2, 16), (1, 0), (2, 0)]
# kind 1 (nbody_forces_batch) keys: mean active rows per system, timed on
# all-active batches of equal systems of this size
BATCH_BUCKETS = [128, 256, 512, 1024, 2048, 4096, 8192, 16384]
# kind 2 (batched block steps) keys: mean system size, timed as
# graph-replayed block steps over one synchronisation interval
STEP_SHAPES = [(1, 1), (1, 4), (1, 16), (1, 64), (1, 0), (2, 0)]
STEP_BUCKETS = [256, 1024, 4096]


def _equal_batch(size, total, seed):
    import synth
    return synth.cluster_batch(seed=seed, n_clusters=max(1, total // size), n_min=size, n_max=size)


def _wall_ms(fn, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def tune_batch_forces(ctx, precisions=("fp64", "mixed", "mixed_ds"), buckets=BATCH_BUCKETS, total=1 << 19,
                      reps=3, log=print):
    """Kind 1 entries: the fastest batched shape for nbody_forces_batch on
    all-active batches of `total` bodies in equal systems of each size (the
    whole call: work list, force kernel and chunk sums)."""
    dev = ctx.device
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    entries = []
    ranges = _midpoints(list(buckets))
    for size, (lo, hi) in zip(buckets, ranges):
        b = _equal_batch(size, total, 11)
        P, V, M = t(b.pos), t(b.vel), t(b.mass)
        n = int(b.offsets[-1])
        act = t(np.arange(n, dtype=np.int32))
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty_like(acc)
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        inter = float(np.sum(b.sizes.astype(np.float64) ** 2))
        for prec in precisions:
            ctx.set_precision(prec)
            best = None
            for K, L in BATCH_SHAPES:
                ctx.tune_clear()
                ctx.tune_add_batch(prec, 1, 1, 2 ** 40, K, L)
                ms = _wall_ms(lambda: ctx.forces_batch(b.offsets, b.eps2, P, V, M, act, b.offsets, acc, jerk, pot),
                              reps)
                if best is None or ms < best[0]:
                    best = (ms, K, L)
            ms, K, L = best
            e = dict(kind=1, prec=prec, key_min=lo, key_max=hi, K=K, L=L, ms=round(ms, 4), rep_size=size,
                     gint=round(inter / ms / 1e6, 1))
            entries.append(e)
            log(json.dumps(e))
    ctx.tune_clear()
    return entries


def tune_batch_steps(ctx, precisions=("fp64", "mixed", "mixed_ds"), buckets=STEP_BUCKETS, total=1 << 18, log=print):
    """Kind 2 entries: the fastest shape for graph-replayed batched block steps
    over one synchronisation interval (dt_max = 1/16) of `total` bodies in
    equal Plummer systems of each size, after a first interval that sizes the
    buffers and captures the graphs."""
    from .integrator import BlockIntegrator
    dev = ctx.device
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    entries = []
    ranges = _midpoints(list(buckets))
    for size, (lo, hi) in zip(buckets, ranges):
        b = _equal_batch(size, total, 12)
        for prec in precisions:
            ctx.set_precision(prec)
            best = None
            for K, L in STEP_SHAPES:
                ctx.tune_clear()
                ctx.tune_add_batch(prec, 2, 1, 2 ** 40, K, L)
                bi = BlockIntegrator(ctx, t(b.pos), t(b.vel), t(b.mass), b.eps2, 0.01, 1.0 / 16, 30,
                                     offsets=b.offsets)
                bi.run_until(1.0 / 16, graph_steps=16)
                torch.cuda.synchronize()
                s0 = bi.steps
                t0 = time.perf_counter()
                bi.run_until(2.0 / 16, graph_steps=16)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3
                if best is None or ms < best[0]:
                    best = (ms, K, L, bi.steps - s0)
                del bi
            ms, K, L, steps = best
            e = dict(kind=2, prec=prec, key_min=lo, key_max=hi, K=K, L=L, ms=round(ms, 3), rep_size=size,
                     steps=int(steps))
            entries.append(e)
            log(json.dumps(e))
    ctx.tune_clear()
    return entries


def forces_source_hash():
    """sha256 of the force kernels' source the table was measured on."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "forces.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def save(entries, path, meta=None):
    doc = {"format": 1, "meta": meta or {}, "entries": entries}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)


def table_path():
    """The launch table a new context installs: the file named by the
    environment variable NB_TUNE_CACHE when it is set, non-empty and exists
    (the autotuner writes there by default); else the shipped table for this
    GPU when it exists (with a warning when NB_TUNE_CACHE names a missing
    file: the cache has not been written yet); else None."""
    env = os.environ.get("NB_TUNE_CACHE", "")
    if env:
        if os.path.exists(env):
            return env
        warnings.warn(f"NB_TUNE_CACHE names {env}, which does not exist yet; using the shipped table",
                      stacklevel=2)
    return DEFAULT_TABLE if os.path.exists(DEFAULT_TABLE) else None


def load(ctx, path=DEFAULT_TABLE):
    """Install a saved table into a context (entries in file order)."""
    with open(path) as f:
        doc = json.load(f)
    single = [e for e in doc["entries"] if e.get("kind", 0) == 0]
    for e in sorted(single, key=lambda e: e["n_min"]):
        ctx.tune_add(e["prec"], e["n_min"], e["act_min"], e["act_max"], e["K"], e["L"], e["items"],
                     e.get("T", 0), e.get("WG", 0))
    for e in doc["entries"]:
        if e.get("kind", 0) in (1, 2):
            ctx.tune_add_batch(e["prec"], e["kind"], e["key_min"], e["key_max"], e["K"], e["L"])
    return len(doc["entries"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[65536, 262144])
    ap.add_argument("--prec", nargs="+", default=["fp64", "mixed", "mixed_ds"])
    ap.add_argument("--out", default=os.environ.get("NB_TUNE_CACHE") or "tuning.json",
                    help="table to write (default: $NB_TUNE_CACHE, else tuning.json)")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--max-active", type=int, default=0,
                    help="largest active-set bucket to time (0: up to N); the top bucket's range then covers every larger count")
    ap.add_argument("--append", default="", help="start from the entries of this table")
    ap.add_argument("--batch", action="store_true", help="also tune the batched kernel (nbody_forces_batch)")
    ap.add_argument("--batch-steps", action="store_true", help="also tune the batched block steps")
    ap.add_argument("--batch-only", action="store_true", help="tune only the batched kernel (no --n sweep)")
    ap.add_argument("--batch-forces-only", action="store_true",
                    help="retune only the batched kernel's entries (nbody_forces_batch); keep every other entry")
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_1409_5474_amd as nb
    ctx = nb.Context(0, "fp64", load_tuning=False)
    t0 = time.time()
    entries = []
    if args.append:
        with open(args.append) as f:
            entries = json.load(f)["entries"]
    buckets = [b for b in BUCKETS if not args.max_active or b <= args.max_active]
    say = lambda m: print(m, flush=True)
    props = torch.cuda.get_device_properties(0)

    def checkpoint():
        # the table so far, after every stage (a long run keeps what it finished)
        save(entries, args.out, meta={"device": props.name, "gcn_arch": getattr(props, "gcnArchName", ""),
                                      "cus": props.multi_processor_count, "seconds": round(time.time() - t0, 1),
                                      "forces_hip_sha256": forces_source_hash()})

    if args.batch_only:
        entries = [e for e in entries if e.get("kind", 0) == 0]
    elif args.batch_forces_only:
        args.batch = True
    else:
        for n in sorted(args.n):
            entries = [e for e in entries if not (e.get("kind", 0) == 0 and e["n_min"] == n)]
            entries += tune(ctx, n, args.prec, buckets=buckets, reps=args.reps, log=say)
            checkpoint()
            print(f"# N={n} done after {time.time() - t0:.0f} s", flush=True)
    if args.batch or args.batch_only:
        entries = [e for e in entries if e.get("kind", 0) != 1]
        entries += tune_batch_forces(ctx, args.prec, reps=args.reps, log=say)
        checkpoint()
        print(f"# batched forces done after {time.time() - t0:.0f} s", flush=True)
    if args.batch_steps or args.batch_only:
        entries = [e for e in entries if e.get("kind", 0) != 2]
        entries += tune_batch_steps(ctx, args.prec, log=say)
        checkpoint()
        print(f"# batched block steps done after {time.time() - t0:.0f} s", flush=True)
    checkpoint()
    print(f"wrote {args.out} ({len(entries)} entries)", flush=True)


if __name__ == "__main__":
    main()
