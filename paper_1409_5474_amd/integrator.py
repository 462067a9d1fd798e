"""Hermite block-step integrator driver (device-resident state, HIP graphs).

The state lives in torch tensors on the GPU; every step runs through the C
ABI's ``nb_block_step`` (schedule -> predict -> forces -> correct, no host
synchronisation).  ``run_until`` captures ``graph_steps`` consecutive block
steps into one HIP graph and replays it; a step beyond the stop time is
empty, so the host reads the schedule once per replay to decide whether to
go on.  The stop time lives in device memory (``nb_set_stop_source``), so one
captured graph serves every later stop time.

Time is kept in integer ticks of dt_max 2^-max_level (see nbody.h).

Metrics (``set_metrics``): a sink -- any callable, e.g. ``jsonl_sink(path)``
-- receives one dict per eager block step (its active count, interactions
and the device time of its three phases) and one per graph replay (steps
and device time); ``run_until(log=...)`` adds one per synchronisation time
(energy, momenta, virial ratio).
"""
import json

import torch

from . import Context

INT64_MAX = 2 ** 63 - 1


def jsonl_sink(path):
    """A metrics sink that appends each record to ``path`` as one JSON line."""
    f = open(path, "a", buffering=1)

    def sink(record):
        f.write(json.dumps(record) + "\n")

    sink.close = f.close
    return sink


class BlockIntegrator:
    """Block-step integration of one system, or of a batch of independent
    systems stored back to back (``offsets`` of length C+1 and one softening
    per system in ``eps2``; the block step is then global over the batch)."""

    metrics = None   # per-step record sink (set_metrics)

    def __init__(self, ctx: Context, pos, vel, mass, eps2, eta=0.01, dt_max=1.0 / 16, max_level=30,
                 offsets=None):
        import numpy as np
        dev = ctx.device
        n = mass.shape[0]
        self.ctx, self.n, self.dev = ctx, n, dev
        self.batch = offsets is not None
        if self.batch:
            self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
            self.eps2_sys = np.ascontiguousarray(eps2, dtype=np.float64)
            if self.offsets[-1] != n or self.eps2_sys.shape[0] != self.offsets.shape[0] - 1:
                raise ValueError("offsets must end at N and eps2 must have one value per system")
            self.eps2 = None
        else:
            self.eps2 = float(eps2)
        self.eta, self.dt_max, self.max_level = float(eta), float(dt_max), int(max_level)
        self.tick = self.dt_max * 2.0 ** -self.max_level
        f64 = dict(dtype=torch.float64, device=dev)
        self.mass = mass.to(**f64).contiguous()
        self.pos = pos.to(**f64).contiguous().clone()
        self.vel = vel.to(**f64).contiguous().clone()
        self.acc = torch.empty((n, 3), **f64)
        self.jerk = torch.empty((n, 3), **f64)
        self.t_tick = torch.zeros(n, dtype=torch.int64, device=dev)
        self.level = torch.zeros(n, dtype=torch.int32, device=dev)
        self.sched = torch.zeros(4, dtype=torch.int64, device=dev)   # t_next, n_active, steps, clamps
        self._alloc_scratch()
        # start-up: forces on every particle at t = 0 and the first levels
        self.restart()
        # the run loops test the earliest particle time on the host; the first
        # such reduction loads its kernel, a one-time cost kept out of the runs
        int(self.t_tick.min().item())

    def _alloc_scratch(self):
        n, dev = self.n, self.dev
        f64 = dict(dtype=torch.float64, device=dev)
        self.stop = torch.full((1,), INT64_MAX, dtype=torch.int64, device=dev)
        self.pos_p = torch.empty((n, 3), **f64)
        self.vel_p = torch.empty((n, 3), **f64)
        self.acc1 = torch.empty((n, 3), **f64)
        self.jerk1 = torch.empty((n, 3), **f64)
        self.pot1 = torch.empty(n, **f64)
        self.active = torch.empty(n, dtype=torch.int32, device=dev)
        self.all_idx = torch.arange(n, dtype=torch.int32, device=dev)
        self._graphs = {}
        self._capturing = False

    def _all_forces(self, pos, vel, acc, jerk, pot):
        if self.batch:
            self.ctx.forces_batch(self.offsets, self.eps2_sys, pos, vel, self.mass, self.all_idx, self.offsets,
                                  acc, jerk, pot)
        else:
            self.ctx.forces(pos, vel, self.mass, self.all_idx, self.eps2, acc, jerk, pot)

    # ---- stepping ---------------------------------------------------------
    def step(self, t_stop_tick=None):
        """One block step on the context stream.  Without ``t_stop_tick`` the
        step stops at the tick held in ``self.stop`` (device memory)."""
        self.ctx.set_stop_source(self.stop if t_stop_tick is None else None)
        try:
            self._step(INT64_MAX if t_stop_tick is None else t_stop_tick)
        finally:
            self.ctx.set_stop_source(None)
        if self.metrics is not None and not self._capturing:
            self._emit_step()

    # ---- metrics ------------------------------------------------------------
    def set_metrics(self, sink):
        """Send per-step records to ``sink`` (a callable taking a dict), or
        stop with None.  Each eager step then waits for the device, so
        metrics are for diagnosis, not for timed runs."""
        self.metrics = sink
        self.ctx.set_phase_timing(sink is not None)

    def _interactions(self, n_act):
        # n_active x N_j, summed per system for a batch
        if not self.batch:
            return n_act * self.n
        import numpy as np
        if n_act == 0:
            return 0
        rows = self.active[:n_act].cpu().numpy()
        sys_of = np.searchsorted(self.offsets, rows, side="right") - 1
        sizes = np.diff(self.offsets)
        return int(sizes[sys_of].sum())

    def _emit_step(self):
        ms = self.ctx.phase_times()
        t_next, n_act, steps, clamps = self.sched.cpu().tolist()
        self.metrics(dict(kind="step", step=steps, t=t_next * self.tick, n_active=n_act,
                          interactions=self._interactions(n_act), ms_schedule=ms[0], ms_forces=ms[1],
                          ms_correct=ms[2], clamps=clamps))

    def _step(self, t_stop_tick):
        if self.batch:
            self.ctx.block_step_batch(self.offsets, self.eps2_sys, self.eta, self.dt_max, self.max_level, self.mass,
                                      self.pos, self.vel, self.acc, self.jerk, self.t_tick, self.level, self.pos_p,
                                      self.vel_p, self.active, self.acc1, self.jerk1, self.pot1, self.sched,
                                      t_stop_tick)
        else:
            self.ctx.block_step(self.n, self.eps2, self.eta, self.dt_max, self.max_level, self.mass, self.pos,
                                self.vel, self.acc, self.jerk, self.t_tick, self.level, self.pos_p, self.vel_p,
                                self.active, self.acc1, self.jerk1, self.pot1, self.sched, t_stop_tick)

    def _graph(self, steps):
        g = self._graphs.get(steps)
        if g is None:
            prev = self.ctx.stream
            stream = torch.cuda.Stream(self.dev)
            self.ctx.set_stream(stream)
            self._capturing = True
            try:
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=stream):
                    for _ in range(steps):
                        self.step()
            finally:
                self._capturing = False
                self.ctx.set_stream(prev)
            self._graphs[steps] = g
        return g

    def run_until(self, t_end, graph_steps=32, use_graph=True, log=None):
        """Integrate until every particle reaches t_end (a multiple of dt_max).
        With ``log`` (a callable), stop at every synchronisation time (each
        multiple of dt_max) on the way and pass it ``diagnostics()``."""
        end = int(round(t_end / self.tick))
        if end * self.tick != t_end:
            raise ValueError("t_end must be a whole number of ticks")
        sync = 1 << self.max_level
        if end % sync:
            raise ValueError("t_end must be a multiple of dt_max (a synchronisation time)")
        if log is None:
            return self.run_to_tick(end, graph_steps, use_graph)
        tick = (int(self.t_tick.min().item()) // sync + 1) * sync
        while tick <= end:
            self.run_to_tick(tick, graph_steps, use_graph)
            log(self.diagnostics())
            tick += sync
        return self

    def restart(self):
        """Start afresh from the current (synchronised) state: forces on every
        particle and start-up levels, as at t = 0 (after an outside change of
        the velocities, e.g. a kick, the stored jerks are stale)."""
        self._all_forces(self.pos, self.vel, self.acc, self.jerk, self.pot1)
        self.ctx.startup(self.acc, self.jerk, self.eta, self.dt_max, self.max_level, self.level)
        self._E0 = self._energy_from(self.pot1)["E"]

    def run_to_tick(self, end, graph_steps=32, use_graph=True):
        """Integrate until every particle reaches tick ``end`` (a multiple of 2^max_level)."""
        end = int(end)
        if end % (1 << self.max_level):
            raise ValueError("t_end must be a multiple of dt_max (a synchronisation time)")
        self.stop.fill_(end)
        # one eager step sizes every workspace before a graph is captured
        self.step()
        while int(self.t_tick.min().item()) < end:
            if use_graph:
                g = self._graph(graph_steps)
                torch.cuda.synchronize(self.dev)
                if self.metrics is not None:
                    s0 = self.steps
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    g.replay()
                    e1.record()
                    torch.cuda.synchronize(self.dev)
                    self.metrics(dict(kind="replay", steps=self.steps - s0, t=self.time,
                                      ms=e0.elapsed_time(e1)))
                else:
                    g.replay()
                torch.cuda.synchronize(self.dev)
            else:
                for _ in range(graph_steps):
                    self.step()
        return self

    # ---- checkpoint / resume ----------------------------------------------
    _STATE = ("pos", "vel", "acc", "jerk", "t_tick", "level", "sched")

    def checkpoint(self, path):
        """Write the integration state to an .npz file (host copies).  The
        kernels are deterministic, so resuming continues bit for bit."""
        import numpy as np
        torch.cuda.synchronize(self.dev)
        arrays = {k: getattr(self, k).cpu().numpy() for k in self._STATE}
        arrays["mass"] = self.mass.cpu().numpy()
        meta = np.array([self.eta, self.dt_max, float(self.max_level), float(self.batch), self._E0], dtype=np.float64)
        arrays["meta"] = meta
        if self.batch:
            arrays["offsets"] = self.offsets
            arrays["eps2_sys"] = self.eps2_sys
        else:
            arrays["eps2"] = np.array([self.eps2], dtype=np.float64)
        np.savez(path, **arrays)

    @classmethod
    def restore(cls, ctx: Context, path):
        """Rebuild an integrator from ``checkpoint`` output."""
        import numpy as np
        d = np.load(path, allow_pickle=False)
        eta, dt_max, max_level, batch, E0 = d["meta"].tolist()
        dev = ctx.device
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self = cls.__new__(cls)
        self.ctx, self.n, self.dev = ctx, int(d["mass"].shape[0]), dev
        self.batch = bool(batch)
        if self.batch:
            self.offsets = d["offsets"].astype(np.int64)
            self.eps2_sys = d["eps2_sys"].astype(np.float64)
            self.eps2 = None
        else:
            self.eps2 = float(d["eps2"][0])
        self.eta, self.dt_max, self.max_level = float(eta), float(dt_max), int(max_level)
        self.tick = self.dt_max * 2.0 ** -self.max_level
        self._E0 = float(E0)
        self.mass = t(d["mass"])
        for k in self._STATE:
            setattr(self, k, t(d[k]))
        for k, v in self._restore_extra(d).items():
            setattr(self, k, v)
        self._alloc_scratch()
        return self

    def _restore_extra(self, d):
        return {}

    # ---- diagnostics ------------------------------------------------------
    @property
    def steps(self):
        return int(self.sched[2].item())

    @property
    def clamps(self):
        return int(self.sched[3].item())

    @property
    def time(self):
        return int(self.t_tick.min().item()) * self.tick

    def energy(self):
        """K, W, E, P, L of the current (synchronised) state, summed over every system."""
        acc = torch.empty_like(self.acc)
        jerk = torch.empty_like(self.jerk)
        pot = torch.empty_like(self.pot1)
        self._all_forces(self.pos, self.vel, acc, jerk, pot)
        return self._energy_from(pot)

    def _energy_from(self, pot):
        out = torch.zeros(8, dtype=torch.float64, device=self.dev)
        self.ctx.energy(self.pos, self.vel, self.mass, pot, out)
        o = out.cpu().tolist()
        return dict(K=o[0], W=o[1], E=o[0] + o[1], P=o[2:5], L=o[5:8])

    @property
    def E0(self):
        """Total energy at the last start (construction or ``restart``)."""
        return self._E0

    def diagnostics(self):
        """The state at a synchronisation time: time, steps so far, clamped
        level changes, energy and its change since the start (``E0``),
        momentum, angular momentum and the virial ratio 2K/|W|."""
        e = self.energy()
        return dict(t=self.time, steps=self.steps, clamps=self.clamps, E=e["E"], K=e["K"], W=e["W"],
                    dE_rel=abs(e["E"] - self._E0) / abs(self._E0) if self._E0 else 0.0, P=e["P"], L=e["L"],
                    virial=2.0 * e["K"] / abs(e["W"]) if e["W"] else float("inf"))


class BlockIntegrator6(BlockIntegrator):
    """Sixth-order Hermite block steps (``nb_block_step6``) of one system.

    Every particle carries a, jdot, snap and crackle; start-up evaluates a and
    jdot, then the snap with those accelerations, sets the crackle to zero and
    takes its levels from dt* = eta_s min(|a|/|j|, sqrt(|a|/|s|)).  ``eta``
    scales the order-six step criterion (typical values 0.1-0.3).  Time,
    levels, graphs, energy and checkpoints work as in ``BlockIntegrator``."""

    _STATE = BlockIntegrator._STATE + ("snap", "crackle")

    def __init__(self, ctx: Context, pos, vel, mass, eps2, eta=0.15, dt_max=1.0 / 16, max_level=30, eta_s=0.01):
        self.eta_s = float(eta_s)
        dev = ctx.device
        n = mass.shape[0]
        self.snap = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        self.crackle = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        super().__init__(ctx, pos, vel, mass, eps2, eta, dt_max, max_level)

    def _alloc_scratch(self):
        super()._alloc_scratch()
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.acc_p = torch.empty((self.n, 3), **f64)
        self.snap1 = torch.empty((self.n, 3), **f64)

    def restart(self):
        """Forces and start-up levels from the current (synchronised) state; crackle = 0."""
        zero = torch.zeros_like(self.acc)
        self.ctx.forces6(self.pos, self.vel, zero, self.mass, self.all_idx, self.eps2, self.acc, self.jerk,
                         self.snap1, self.pot1)
        self.ctx.forces6(self.pos, self.vel, self.acc, self.mass, self.all_idx, self.eps2, self.acc1, self.jerk,
                         self.snap, self.pot1)
        self.acc.copy_(self.acc1)
        self.crackle.zero_()
        self.ctx.startup6(self.acc, self.jerk, self.snap, self.eta_s, self.dt_max, self.max_level, self.level)
        self._E0 = self._energy_from(self.pot1)["E"]

    def _step(self, t_stop_tick):
        self.ctx.block_step6(self.n, self.eps2, self.eta, self.dt_max, self.max_level, self.mass, self.pos, self.vel,
                             self.acc, self.jerk, self.snap, self.crackle, self.t_tick, self.level, self.pos_p,
                             self.vel_p, self.acc_p, self.active, self.acc1, self.jerk1, self.snap1, self.pot1,
                             self.sched, t_stop_tick)

    def checkpoint(self, path):
        import numpy as np
        super().checkpoint(path)
        d = dict(np.load(path, allow_pickle=False))
        d["eta_s"] = np.array([self.eta_s])
        np.savez(path, **d)

    def _restore_extra(self, d):
        self.eta_s = float(d["eta_s"][0])
        return {}
