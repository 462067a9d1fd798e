"""Benchmark: direct-summation acc+jerk(+pot) throughput on one MI355X.

Workload: Plummer sphere, N = 262144 (2^18), equal masses, eps = 1/256,
mixed precision (double-precision separations, float pair arithmetic,
double accumulation), every particle active.  One step = one Hermite block
step through the library's block-step entry point: schedule, predict all
N particles, forces on the active set (all N), correct.  The run uses one
step level, so every block step has all N particles active (a
shared-time-step Hermite step); N^2 pair interactions per step.

Printed: one JSON line with the metric (G-interactions/s of the whole step,
mixed precision), the FP64 figure and the mixed/FP64 speedup on the same
GPU, the roofline of the force kernel (VALU-bound; nominal 43 flops per
interaction against the FP32 vector peak), and the CPU oracle's rate on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_INTERACTION = 43          # nominal count for acc + jerk + pot
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_kernel_hbm_traffic.md")
FORCE_SRC = os.path.join(ROOT, "paper_1409_5474_amd", "csrc", "forces.hip")
FP32_VECTOR_PEAK_TFLOPS = 157.3     # MI355X, vendor figure
FP64_VECTOR_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=262144)
    ap.add_argument("--prec", default="mixed", choices=["mixed", "mixed_ds", "fp64"])
    ap.add_argument("--force-only", action="store_true",
                    help="profiling target: only the all-active force launch, --steps times")
    ap.add_argument("--kernel", default="direct", choices=["direct", "snap", "tree"],
                    help="with --force-only: the direct force kernel, the sixth-order snap kernel (FP64) or the tree "
                         "code (theta=0.5; FP64 or mixed force terms with --prec)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="profiling target: a plain device-to-device copy of this many bytes, --steps times "
                         "(calibrates the HBM byte counters)")
    ap.add_argument("--workload", default="", choices=["", "plummer1k", "hermite65k", "hermite262k", "batch128",
                                                        "merger", "bridge", "hermite6", "tree", "passes"],
                    help="instead of the headline line, measure one of the other workloads (see workloads())")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    return ap.parse_args()


def measured_traffic(prec):
    """HBM bytes per launch of the all-active force kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel source
    has changed since those counters were taken (or none were taken)."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
        src = hashlib.sha256(open(FORCE_SRC, "rb").read()).hexdigest()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith("traffic-json:"):
            d = json.loads(ln.split(":", 1)[1])
            if d.get("forces_hip_sha256") == src and d.get("prec") == prec:
                return d.get("hbm_bytes_per_launch")
    return None


def spread(xs):
    """Median, minimum and maximum of a list of times (ms)."""
    ys = sorted(xs)
    m = len(ys) // 2
    med = ys[m] if len(ys) % 2 else 0.5 * (ys[m - 1] + ys[m])
    return {"median": round(med, 4), "min": round(ys[0], 4), "max": round(ys[-1], 4)}


# vector-ISA flags that bear on the oracle's speed
CPU_ISA_FLAGS = ("sse4_2", "avx", "avx2", "fma", "avx512f", "avx512dq", "avx512vl", "avx512_bf16")


def cpu_model():
    """The host CPU's model name, logical CPU count, threads per core and the
    vector-ISA flags among CPU_ISA_FLAGS that it reports, from lscpu."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    info = {}
    for ln in out.splitlines():
        k, _, v = ln.partition(":")
        info[k.strip()] = v.strip()
    flags = set(info.get("Flags", "").split())
    return {"model": info.get("Model name"), "logical_cpus": info.get("CPU(s)"),
            "threads_per_core": info.get("Thread(s) per core"),
            "isa_flags": [f for f in CPU_ISA_FLAGS if f in flags]}


class ClockSampler:
    """Samples the GPU's graphics clocks with amd-smi in a background thread
    while the timed runs go on (one sample = the mean over the GPU's dies);
    summary() gives the median and range of the samples taken while kernels
    ran (None when amd-smi is not available)."""

    def __init__(self, period=0.5):
        import threading
        self.period, self.samples, self._stop = period, [], threading.Event()
        self._t = threading.Thread(target=self._loop, daemon=True)

    def _loop(self):
        import re
        import subprocess
        while not self._stop.is_set():
            try:
                out = subprocess.run(["amd-smi", "metric", "-g", "0", "-c"], capture_output=True, text=True,
                                     timeout=10).stdout
            except (OSError, subprocess.SubprocessError):
                return
            mhz = [int(x) for x in re.findall(r"GFX_\d+:\s*\n\s*CLK: (\d+) MHz", out)]
            if mhz:
                self.samples.append(sum(mhz) / len(mhz))
            self._stop.wait(self.period)

    def start(self):
        self._t.start()

    def stop(self):
        self._stop.set()
        self._t.join(timeout=15)

    def summary(self):
        busy = [x for x in self.samples if x > 1000]   # samples taken while kernels ran
        if not busy:
            return None
        d = spread(busy)
        d["samples"] = len(busy)
        return d


def workloads(args):
    """Measurements of the other workloads (one JSON line each).

    plummer1k   Plummer N=1024, eps=0.01, FP64, one all-active evaluation
    hermite65k  Plummer N=65536, eps=1/256, FP64 Hermite block steps (eta=0.01,
                dt_max=1/16) to t=1/8, graph-replayed; energy drift, steps
    hermite262k Plummer N=262144, eps=1/256, block steps to t=1/8 in FP64 and
                in mixed precision: drift of each and the time of each.  Both
                Hermite workloads also report the active-set sizes and the
                interactions (sum of n_active x N, from an untimed eager replay
                of the FP64 run) and the effective rate over the timed run
    batch128    128 Plummer clusters, N log-uniform in [128, 16384],
                eps_c = 0.05 N_c^-1/3, mixed, block steps to t=1/16, one
                graph replay per 8 steps vs eager launches
    merger      11 Hernquist galaxies (2^17 stars + a point mass each): the
                i-set near the point masses against all 1,441,803 bodies,
                FP64 and mixed
    hermite6    sixth-order Hermite: the snap kernel on Plummer N=262144 all
                active (FP64), and block steps of Plummer N=65536, eps=1/256,
                to t=1/8 (eta=0.4, eta_s=0.02, graph-replayed) beside the
                fourth-order run of the same model (eta=0.01): steps, time
                and energy drift of each
    tree        the Barnes-Hut tree code on Plummer spheres of 2^18 and 2^20
                particles (eps=1/256, n_crit=16, groups of 64), FP64 and
                mixed force terms: wall time of one force evaluation for
                theta = 0.75, 0.5, 0.4 (the call includes the build),
                interaction pairs, and the acceleration error against FP64
                direct sums on 4096 sampled particles
    bridge      the same bodies under the kick-drift-kick split: c = the
                point masses and the stars near them (FP64 Hermite block
                steps, eta=0.01), g = every other star (leapfrog with the
                mixed-precision tree code at theta=0.5 -- the paper's hybrid
                -- or with mixed-precision direct forces), cross field in mixed
                precision, direct both ways or (tree_cross) the field of g on c
                from the tree evaluation; bridge step 1/128; --steps bridge
                steps after one warm-up step, each part timed
    passes      the HBM-bound passes of a block step on 2^22 particles (all
                active): predictor, corrector, scheduler, energy sums, kick
                and kick-drift; HIP events over --steps launches of each; the
                algorithmic bytes per particle (every array the pass must read
                or write, once) over the mean launch time, against the 8 TB/s
                HBM peak
    """
    import numpy as np
    import torch

    import paper_1409_5474_amd as nb
    import synth
    from paper_1409_5474_amd.integrator import BlockIntegrator

    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {"workload": args.workload, "data": "synthetic (seeded)"}
    if args.workload == "plummer1k":
        p = synth.plummer(1024, 1)
        ctx = nb.Context(0, "fp64")
        act = torch.arange(1024, dtype=torch.int32, device=dev)
        P, V, M = t(p.pos), t(p.vel), t(p.mass)
        ctx.forces(P, V, M, act, 1e-4)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(args.steps):
            ctx.forces(P, V, M, act, 1e-4)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out.update(n=1024, prec="fp64", ms_per_eval=round(ms, 5), gint=round(1024 * 1024 / ms / 1e6, 3))
    elif args.workload in ("hermite65k", "hermite262k"):
        n, seed = (65536, 2) if args.workload == "hermite65k" else (262144, 3)
        p = synth.plummer(n, seed)
        precs = ("fp64",) if n == 65536 else ("fp64", "mixed")
        for prec in precs:
            ctx = nb.Context(0, prec)
            bi = BlockIntegrator(ctx, t(p.pos), t(p.vel), t(p.mass), 2.0 ** -16, 0.01, 1.0 / 16, 30)
            E0 = bi.energy()["E"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bi.run_until(0.125, graph_steps=32)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            E1 = bi.energy()
            evals = None
            out[prec] = dict(n=n, steps=bi.steps, clamps=bi.clamps, wall_s=round(wall, 3),
                             E0=E0, E1=E1["E"], drift=abs(E1["E"] - E0) / abs(E0),
                             level_histogram=np.bincount(bi.level.cpu().numpy(), minlength=31).tolist())
            if prec == precs[0]:
                # untimed eager replay of the same run: the active-set sizes of every step
                bc = BlockIntegrator(ctx, t(p.pos), t(p.vel), t(p.mass), 2.0 ** -16, 0.01, 1.0 / 16, 30)
                end = int(round(0.125 / bc.tick))
                bc.stop.fill_(end)
                sizes = []
                while int(bc.t_tick.min().item()) < end:
                    bc.step()
                    sizes.append(int(bc.sched[1].item()))
                sizes = np.array(sizes, dtype=np.int64)
                active_stats = dict(steps=len(sizes), mean_active=round(float(sizes.mean()), 1),
                                    median_active=int(np.median(sizes)), max_active=int(sizes.max()),
                                    interactions=int(sizes.sum()) * n)
            out[prec].update(active_stats)
            out[prec]["gint_effective"] = round(active_stats["interactions"] / wall / 1e9, 1)
            if n == 65536:
                out[prec]["pos_sample"] = bi.pos.cpu().numpy()[::4096].tolist()
            ctx.close()
    elif args.workload == "batch128":
        b = synth.cluster_batch(seed=4, n_clusters=128)
        ctx = nb.Context(0, "mixed")
        res = {}
        for mode in ("graph", "eager"):
            bi = BlockIntegrator(ctx, t(b.pos), t(b.vel), t(b.mass), b.eps2, 0.01, 1.0 / 16, 30, offsets=b.offsets)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bi.run_until(0.0625, graph_steps=8, use_graph=(mode == "graph"))
            torch.cuda.synchronize()
            res[mode] = dict(wall_s=round(time.perf_counter() - t0, 3), steps=bi.steps)
        # one all-active batched evaluation: interactions = sum N_c^2
        n = int(b.offsets[-1])
        act = torch.arange(n, dtype=torch.int32, device=dev)
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        jerk, pot = torch.empty_like(acc), torch.empty(n, dtype=torch.float64, device=dev)
        P, V, M = t(b.pos), t(b.vel), t(b.mass)
        ctx.forces_batch(b.offsets, b.eps2, P, V, M, act, b.offsets, acc, jerk, pot)
        # back-to-back calls: each plans its work list on the host while the
        # previous one runs, but the first timed call's planning precedes its
        # launch, so a few calls alone would understate the steady rate
        reps = max(args.steps, 20)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(reps):
            ctx.forces_batch(b.offsets, b.eps2, P, V, M, act, b.offsets, acc, jerk, pot)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        inter = float((b.sizes.astype(np.float64) ** 2).sum())
        out.update(clusters=128, bodies=n, interactions_all_active=inter, calls_all_active=reps, ms_all_active=round(ms, 4),
                   gint_all_active=round(inter / ms / 1e6, 2), block_steps_to_t_1_16=res,
                   graph_speedup=round(res["eager"]["wall_s"] / res["graph"]["wall_s"], 3))
    elif args.workload == "merger":
        m = synth.hernquist_merger()
        P, V, M = t(m.pos), t(m.vel), t(m.mass)
        act = t(m.active)
        for prec in ("fp64", "mixed"):
            ctx = nb.Context(0, prec)
            ctx.forces(P, V, M, act, m.eps2)
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(args.steps):
                ctx.forces(P, V, M, act, m.eps2)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            na, nj = int(m.active.size), int(m.mass.size)
            out[prec] = dict(n_i=na, n_j=nj, ms=round(ms, 4), gint=round(na * nj / ms / 1e6, 2),
                             launch=ctx.get_launch(nj, na))
            ctx.close()
    elif args.workload == "hermite6":
        from paper_1409_5474_amd.integrator import BlockIntegrator6
        ctx = nb.Context(0, "fp64")
        n = 262144
        p = synth.plummer(n, 3)
        P, V, M = t(p.pos), t(p.vel), t(p.mass)
        act = torch.arange(n, dtype=torch.int32, device=dev)
        A, J, _ = ctx.forces(P, V, M, act, 2.0 ** -16)
        outs = [torch.empty((n, 3), dtype=torch.float64, device=dev) for _ in range(3)]
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        ctx.forces6(P, V, A, M, act, 2.0 ** -16, *outs, pot)
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(args.steps):
            ctx.forces6(P, V, A, M, act, 2.0 ** -16, *outs, pot)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out["snap_kernel"] = dict(n=n, prec="fp64", ms=round(ms, 3), gint=round(float(n) * n / ms / 1e6, 1))
        n2 = 65536
        p2 = synth.plummer(n2, 2)
        runs = {}
        for order in (4, 6):
            if order == 4:
                bi = BlockIntegrator(ctx, t(p2.pos), t(p2.vel), t(p2.mass), 2.0 ** -16, 0.01, 1.0 / 16, 30)
            else:
                bi = BlockIntegrator6(ctx, t(p2.pos), t(p2.vel), t(p2.mass), 2.0 ** -16, 0.4, 1.0 / 16, 30, 0.02)
            E0 = bi.energy()["E"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bi.run_until(0.125, graph_steps=32)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            E1 = bi.energy()["E"]
            runs[f"order{order}"] = dict(steps=bi.steps, wall_s=round(wall, 3), drift=abs(E1 - E0) / abs(E0))
        out["plummer65k_to_t_1_8"] = runs
        ctx.close()
    elif args.workload == "passes":
        n = 1 << 22
        g = torch.Generator(device=dev).manual_seed(7)
        rnd = lambda *shape: torch.rand(*shape, generator=g, dtype=torch.float64, device=dev)
        ctx = nb.Context(0, "fp64")
        pos, vel, acc, jerk = rnd(n, 3), rnd(n, 3), rnd(n, 3), rnd(n, 3)
        pos_p, vel_p, acc1, jerk1 = rnd(n, 3), rnd(n, 3), rnd(n, 3), rnd(n, 3)
        mass, pot = rnd(n) + 1.0, -rnd(n)
        max_level, dt_max = 30, 1.0 / 16
        level = torch.full((n,), 10, dtype=torch.int32, device=dev)
        t_tick = torch.zeros(n, dtype=torch.int64, device=dev)
        active = torch.arange(n, dtype=torch.int32, device=dev)
        sched = torch.zeros(4, dtype=torch.int64, device=dev)
        eout = torch.zeros(8, dtype=torch.float64, device=dev)
        tick = dt_max * 2.0 ** -max_level
        # bytes per particle: predictor x, v, a, j, t read, x_p, v_p written; corrector (every
        # particle in the active list; the values only move levels and ticks) index, level, t,
        # a, j, x_p, v_p, a1, j1 read, x, v, a, j, t, level written; scheduler three passes
        # over t and level, index written per active particle; energy x, v, m, phi; kick v read
        # and written, a read; kick-drift x and v read and written, a read
        passes = {
            "predict": (152, lambda: ctx.predict(pos, vel, acc, jerk, t_tick, 1 << 20, tick, pos_p, vel_p)),
            "correct": (268, lambda: ctx.correct(active, pos_p, vel_p, acc1, jerk1, pos, vel, acc, jerk, t_tick,
                                                 level, 0.01, dt_max, max_level)),
            "schedule": (40, lambda: ctx.schedule(t_tick, level, max_level, active, sched)),
            "energy": (64, lambda: ctx.energy(pos, vel, mass, pot, eout)),
            "kick": (72, lambda: ctx.kick(vel_p, acc1, 1e-9)),
            "kick_drift": (120, lambda: ctx.kick_drift(pos_p, vel_p, acc1, 1e-9, 1e-9)),
        }
        res = {}
        for name, (bpp, fn) in passes.items():
            fn()
            torch.cuda.synchronize()
            reps = max(1, args.steps)
            e0, e1 = ev(), ev()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if name == "schedule":
                # three reads of t and level, and the index of each active particle
                bpp = 36 + 4 * int(sched[1].item()) / n
            res[name] = dict(bytes_per_particle=round(bpp, 2), ms=round(ms, 4), gb_s=round(bpp * n / ms / 1e6, 1),
                             frac_of_8tbs=round(bpp * n / ms / 1e6 / 8000.0, 3))
        out.update(n=n, passes=res)
        ctx.close()
    elif args.workload == "tree":
        res = {}
        ctx = nb.Context(0, "fp64")
        cmx = nb.Context(0, "mixed")
        for n in (262144, 1048576):
            p = synth.plummer(n, 3)
            P, V, M = t(p.pos), t(p.vel), t(p.mass)
            sample = torch.from_numpy(np.linspace(0, n - 1, 4096).astype(np.int32)).to(dev)
            a_ref, _, _ = ctx.forces(P, V, M, sample, 2.0 ** -16)
            a_ref = a_ref.cpu().numpy()
            for prec, cx in (("fp64", ctx), ("mixed", cmx)):
                for theta in (0.75, 0.5, 0.4):
                    # warm-up with the counts (synchronises), then timed calls without them
                    acc, pot, st = cx.tree_forces(P, M, 2.0 ** -16, theta, 16, 1.0 / 16)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(args.steps):
                        cx.tree_forces(P, M, 2.0 ** -16, theta, 16, 1.0 / 16, acc=acc, pot=pot, stats=False)
                    torch.cuda.synchronize()
                    wall = (time.perf_counter() - t0) / args.steps
                    # the same evaluation replayed from a graph (nothing read on the host)
                    gs = torch.cuda.Stream(dev)
                    cx.set_stream(gs)
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=gs):
                        cx.tree_forces(P, M, 2.0 ** -16, theta, 16, 1.0 / 16, acc=acc, pot=pot, stats=False)
                    cx.set_stream(None)
                    torch.cuda.synchronize()
                    with torch.cuda.stream(gs):
                        g.replay()
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(gs)
                        for _ in range(args.steps):
                            g.replay()
                        e1.record(gs)
                    torch.cuda.synchronize()
                    ms_graph = e0.elapsed_time(e1) / args.steps
                    del g
                    cx.sync()
                    a = acc[sample].cpu().numpy()
                    rel = np.linalg.norm(a - a_ref, axis=1) / np.linalg.norm(a_ref, axis=1)
                    res[f"N{n}_theta{theta}_{prec}"] = dict(ms=round(1e3 * wall, 2), ms_graph=round(ms_graph, 2),
                                                            particles_per_s=round(n / wall, 0),
                                                            acc_rel_err_rms=float(np.sqrt(np.mean(rel ** 2))),
                                                            acc_rel_err_max=float(rel.max()), **st)
        out.update(res)
        ctx.close()
        cmx.close()
    elif args.workload == "bridge":
        from paper_1409_5474_amd.bridge import Bridge
        m = synth.hernquist_merger()
        is_c = np.zeros(m.mass.size, dtype=bool)
        is_c[m.active] = True
        c, g = np.nonzero(is_c)[0], np.nonzero(~is_c)[0]
        dt = 1.0 / 128
        ng, nc = int(g.size), int(c.size)
        out.update(n_g=ng, n_c=nc, bridge_dt=dt, bridge_steps=args.steps)
        for name, field, xfield in (("tree", "tree", "direct"), ("tree_cross", "tree", "tree"),
                                    ("direct", "direct", "direct")):
            c64, cmx = nb.Context(0, "fp64"), nb.Context(0, "mixed")
            # the field (tree or direct sum) and the cross field in mixed precision, the cluster in FP64
            br = Bridge(c64, cmx, t(m.pos[g]), t(m.vel[g]), t(m.mass[g]), t(m.pos[c]),
                        t(m.vel[c]), t(m.mass[c]), m.eps2, m.eps2, m.eps2, dt, n_sub=1, eta=0.01, max_level=30,
                        ctx_x=cmx, field=field, theta=0.5, cross=xfield)
            E0 = br.energy()
            parts = dict(kick=0.0, cluster=0.0, galaxy=0.0)
            block_steps = 0

            def timed(key, fn):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                parts[key] += time.perf_counter() - t0

            for k in range(args.steps + 1):
                if k == 1:                      # the first step is the warm-up
                    parts = dict(kick=0.0, cluster=0.0, galaxy=0.0)
                    block_steps = br.block_steps
                timed("kick", lambda: br.kick(0.5 * dt))
                timed("cluster", br.drift_cluster)
                timed("galaxy", br.drift_galaxy)
                timed("kick", lambda: br.kick(0.5 * dt))
                br.steps += 1
            E1 = br.energy()
            nsteps = args.steps
            wall = sum(parts.values())
            # both directions once (the closing kick's field serves the next opening kick);
            # with the tree giving the field of g on c, only the field of c on g is a direct sum
            cross = (1.0 if xfield == "tree" else 2.0) * ng * nc
            out[name] = dict(ms_per_bridge_step=round(1e3 * wall / nsteps, 2),
                              ms_per_part={k: round(1e3 * v / nsteps, 2) for k, v in parts.items()},
                              cross_field_gint=round(cross * nsteps / parts["kick"] / 1e9, 1),
                              cluster_block_steps_per_bridge_step=round((br.block_steps - block_steps) / nsteps, 1),
                              energy_drift=abs(E1["E"] - E0["E"]) / abs(E0["E"]), time=br.time)
            if field == "direct":
                out[name]["galaxy_gint"] = round(float(ng) * ng * nsteps / parts["galaxy"] / 1e9, 1)
            c64.close(); cmx.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload:
        return workloads(args)
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1409_5474_amd as nb
    import synth

    dev = torch.device("cuda", 0)
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": args.warmup + args.steps}), flush=True)
        return
    if args.force_only:
        p = synth.plummer(args.n, 3)
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        ctx = nb.Context(0, args.prec)
        P, V, M = t(p.pos), t(p.vel), t(p.mass)
        act = torch.arange(args.n, dtype=torch.int32, device=dev)
        acc = torch.empty((args.n, 3), dtype=torch.float64, device=dev)
        jerk, pot = torch.empty_like(acc), torch.empty(args.n, dtype=torch.float64, device=dev)
        if args.kernel == "snap":
            snap = torch.empty_like(acc)
            ctx.forces(P, V, M, act, 2.0 ** -16, acc, jerk, pot)
            A = acc.clone()
            for _ in range(args.warmup + args.steps):
                ctx.forces6(P, V, A, M, act, 2.0 ** -16, acc, jerk, snap, pot)
        elif args.kernel == "tree":
            for _ in range(args.warmup + args.steps):
                ctx.tree_forces(P, M, 2.0 ** -16, 0.5, 16, 1.0 / 16, acc, pot)
        else:
            for _ in range(args.warmup + args.steps):
                ctx.forces(P, V, M, act, 2.0 ** -16, acc, jerk, pot)
        torch.cuda.synchronize()
        print(json.dumps({"force_only": args.prec, "kernel": args.kernel, "n": args.n,
                          "launches": args.warmup + args.steps,
                          "launch_KLS": ctx.get_launch(args.n, args.n)}), flush=True)
        return
    n = args.n
    eps2 = 2.0 ** -16
    p = synth.plummer(n, 3)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    mass = t(p.mass)
    stream = torch.cuda.current_stream(dev)

    def make_state():
        st = dict(pos=t(p.pos), vel=t(p.vel))
        st["acc"] = torch.empty((n, 3), dtype=torch.float64, device=dev)
        st["jerk"] = torch.empty_like(st["acc"])
        st["t_tick"] = torch.zeros(n, dtype=torch.int64, device=dev)
        st["level"] = torch.zeros(n, dtype=torch.int32, device=dev)
        st["pos_p"] = torch.empty_like(st["acc"])
        st["vel_p"] = torch.empty_like(st["acc"])
        st["active"] = torch.empty(n, dtype=torch.int32, device=dev)
        st["acc1"] = torch.empty_like(st["acc"])
        st["jerk1"] = torch.empty_like(st["acc"])
        st["pot1"] = torch.empty(n, dtype=torch.float64, device=dev)
        st["sched"] = torch.zeros(4, dtype=torch.int64, device=dev)
        return st

    dt_max, max_level, eta = 2.0 ** -12, 0, 0.01

    def run(prec):
        ctx = nb.Context(0, prec)
        st = make_state()
        act = torch.arange(n, dtype=torch.int32, device=dev)
        # start-up forces at t = 0 for every particle
        ctx.forces(st["pos"], st["vel"], mass, act, eps2, st["acc"], st["jerk"], st["pot1"])

        def step():
            ctx.block_step(n, eps2, eta, dt_max, max_level, mass, st["pos"], st["vel"], st["acc"], st["jerk"],
                           st["t_tick"], st["level"], st["pos_p"], st["vel_p"], st["active"], st["acc1"],
                           st["jerk1"], st["pot1"], st["sched"])

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # one event before every step and one after the last: the mean over the
        # whole timed region, plus the spread of single steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for k in range(args.steps):
            step()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
        ms_step = ev[0].elapsed_time(ev[-1]) / args.steps
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sched = st["sched"].cpu().tolist()
        assert sched[1] == n, f"block step was not all-active: {sched}"
        # the force kernel alone, same inputs and launch, HIP events on its stream
        acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
        jerk = torch.empty_like(acc)
        pot = torch.empty(n, dtype=torch.float64, device=dev)
        ctx.forces(st["pos_p"], st["vel_p"], mass, act, eps2, acc, jerk, pot)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            ctx.forces(st["pos_p"], st["vel_p"], mass, act, eps2, acc, jerk, pot)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_force = e0.elapsed_time(e1) / args.steps
        launch = ctx.get_launch(n, n)
        finite = bool(torch.isfinite(st["pos"]).all().item())
        ctx.close()
        return dict(ms_step=ms_step, wall_s=wall, ms_force=ms_force, launch=launch, sched=sched, finite=finite,
                    step_ms=spread(per_step))

    clocks = ClockSampler()
    clocks.start()
    res = {args.prec: run(args.prec)}
    other = "fp64" if args.prec == "mixed" else "mixed"
    res[other] = run(other)
    clocks.stop()
    main_r = res[args.prec]
    inter = float(n) * float(n)
    value = inter / (main_r["ms_step"] * 1e-3) / 1e9
    fp64_gint = inter / (res["fp64"]["ms_step"] * 1e-3) / 1e9
    mixed_gint = inter / (res["mixed"]["ms_step"] * 1e-3) / 1e9
    achieved = FLOPS_PER_INTERACTION * inter / (main_r["ms_force"] * 1e-3) / 1e12
    peak = FP32_VECTOR_PEAK_TFLOPS if args.prec == "mixed" else FP64_VECTOR_PEAK_TFLOPS

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        probe = np.arange(0, n, n // 256, dtype=np.int32)[:256]
        t0 = time.perf_counter()
        oracle.forces_f64(p.pos, p.vel, p.mass, eps2, probe, nthreads=threads)
        rate = 256 * n / (time.perf_counter() - t0)
        rows = int(min(n, max(256, args.cpu_seconds * rate / n)))
        sample = np.linspace(0, n - 1, rows).astype(np.int32)
        t0 = time.perf_counter()
        oracle.forces_f64(p.pos, p.vel, p.mass, eps2, sample, nthreads=threads)
        dt = time.perf_counter() - t0
        from oracle import build as oracle_build
        cpu = {"value": rows * n / dt / 1e9, "unit": "G-interactions/s", "cores": threads, "kind": "oracle",
               "sample": f"{rows} evenly spaced i-rows of the N={n} Plummer workload against all {n} j "
                         f"(FP64 oracle, {dt:.1f} s)",
               "cpu_model": cpu_model(), "compiler_flags": "gcc " + " ".join(oracle_build.CFLAGS)}

    line = {
        "metric": "G-interactions/s (acc+jerk) and % vector peak at N=262144; mixed vs FP64",
        "value": round(value, 2),
        "unit": "G-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair / f64 separation+accumulation" if args.prec == "mixed" else "f64",
        "data": "synthetic (seeded Plummer sphere)",
        "config": {"workload": f"Plummer N={n}, eps=1/256, all particles active, shared-step Hermite block step "
                               f"({args.prec})", "n": n, "eps2": eps2, "launch_KLS": main_r["launch"]},
        "fp64": {"value": round(fp64_gint, 2), "ms_per_step": round(res["fp64"]["ms_step"], 4),
                 "ms_force_kernel": round(res["fp64"]["ms_force"], 4),
                 "pct_fp64_vector_peak": round(100 * FLOPS_PER_INTERACTION * inter /
                                               (res["fp64"]["ms_force"] * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 2)},
        "mixed": {"value": round(mixed_gint, 2), "ms_per_step": round(res["mixed"]["ms_step"], 4),
                  "ms_force_kernel": round(res["mixed"]["ms_force"], 4),
                  "pct_fp32_vector_peak": round(100 * FLOPS_PER_INTERACTION * inter /
                                                (res["mixed"]["ms_force"] * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 2)},
        "mixed_vs_fp64_speedup": round(res["fp64"]["ms_step"] / res["mixed"]["ms_step"], 3),
        "step_ms": main_r["step_ms"],
        "gpu_clock_mhz": clocks.summary(),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 4), "traffic": measured_traffic(args.prec),
                     "kernel": f"force kernel ({args.prec}), {FLOPS_PER_INTERACTION} flops x N^2 per launch",
                     "ms_per_launch": round(main_r["ms_force"], 4)},
        "cpu_baseline": cpu,
        "finite": all(r["finite"] for r in res.values()),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
