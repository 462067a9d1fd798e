"""Second-order Hamiltonian split of a collisional subsystem and a field
subsystem, on the GPU (section "The multi-scale approach").

H = H_A + H_B with H_A = W_gc, the potential energy between the field
particles g and the collisional particles c (the stars in the sphere of
influence of the central black holes), and H_B = H_g + H_c.  One step of
length dt is e^{dt/2 A} e^{dt B} e^{dt/2 A}:

  kick(dt/2)  both subsystems take the other's field at the current
              positions: ``nbody_forces_ij`` both ways, then ``nb_kick``;
  drift(dt)   c: the Hermite block-step integrator (``BlockIntegrator``),
              restarted -- new forces and start-up levels -- since the kick
              changed its velocities, with dt_max = dt, so each drift ends on
              a synchronisation time;
              g: n_sub shared-step leapfrog substeps of dt/n_sub with its own
              forces (``nb_kick_drift``, the field solver, ``nb_kick``): the
              paper's tree code (``field="tree"``, ``nb_tree_forces``) or the
              direct sum (``field="direct"``, ``nbody_forces``);
  kick(dt/2).

The closing kick of one step and the opening kick of the next see the same
positions, so the cross field computed for the first serves the second
(kicks change velocities only); any drift invalidates it.

Cross field: ``cross="direct"`` sums both directions directly
(``nbody_forces_ij``).  ``cross="tree"`` (with ``field="tree"``) lets each
subsystem's solver give the field it exerts, as when the two codes of the
paper's hybrid are coupled: the field of g on c comes from the tree code,
evaluated together with g's own forces on the combined set [g | c] with the
masses of c set to zero, and the field of c on g is the direct sum over c.
It needs eps2_gc == eps2_g (one tree evaluation serves both).

Every arithmetic step runs in the library's kernels; this module only
sequences the calls on the contexts' streams.  The subsystems may use
different contexts (and so precisions): ``ctx_c`` for c, ``ctx_g`` for g's
own forces, ``ctx_x`` for the cross field (default ``ctx_g``).  All contexts
must be on the same device and use the same stream (torch's current one by
default).
"""
import torch

from . import Context
from .integrator import BlockIntegrator


class Bridge:
    def __init__(self, ctx_c: Context, ctx_g: Context, xg, vg, mg, xc, vc, mc, eps2_g, eps2_c, eps2_gc, dt,
                 n_sub=1, eta=0.01, max_level=30, ctx_x: Context = None, field="direct", theta=0.5, n_crit=16,
                 g_frac=1.0 / 16, cross="direct"):
        if field not in ("direct", "tree"):
            raise ValueError("field must be 'direct' or 'tree'")
        if cross not in ("direct", "tree"):
            raise ValueError("cross must be 'direct' or 'tree'")
        if cross == "tree" and (field != "tree" or float(eps2_gc) != float(eps2_g)):
            raise ValueError("cross='tree' needs field='tree' and eps2_gc == eps2_g")
        self.field, self.theta, self.n_crit, self.g_frac = field, float(theta), int(n_crit), float(g_frac)
        self.cross = cross
        self.ctx_c, self.ctx_g = ctx_c, ctx_g
        self.ctx_x = ctx_x if ctx_x is not None else ctx_g
        dev = ctx_c.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.eps2_g, self.eps2_c, self.eps2_gc = float(eps2_g), float(eps2_c), float(eps2_gc)
        self.dt, self.n_sub, self.steps = float(dt), int(n_sub), 0
        self.vg = vg.to(**f64).contiguous().clone()
        self.mg = mg.to(**f64).contiguous()
        self.ng = self.mg.shape[0]
        self.cluster = BlockIntegrator(ctx_c, xc, vc, mc, eps2_c, eta, self.dt, max_level)
        self.nc = self.cluster.n
        self.idx_g = torch.arange(self.ng, dtype=torch.int32, device=dev)
        self.idx_c = torch.arange(self.nc, dtype=torch.int32, device=dev)
        if cross == "tree":
            # g's positions and accelerations, and the field of g at c, are
            # views of the combined [g | c] arrays of the tree evaluation
            self._xgc = torch.empty((self.ng + self.nc, 3), **f64)
            self._xgc[:self.ng] = xg.to(**f64)
            self._mgc = torch.cat([self.mg, torch.zeros(self.nc, **f64)])
            self._agc = torch.zeros((self.ng + self.nc, 3), **f64)
            self._pgc = torch.empty(self.ng + self.nc, **f64)
            self.xg = self._xgc[:self.ng]
            self.ag = self._agc[:self.ng]
            self.a_cg = self._agc[self.ng:]
        else:
            self.xg = xg.to(**f64).contiguous().clone()
            self.ag = torch.zeros((self.ng, 3), **f64)
            self.a_cg = torch.empty((self.nc, 3), **f64)
        self._tree_cg_valid = False  # the tree's field of g on c belongs to the current positions
        self._jg = torch.empty((self.ng, 3), **f64)
        self._pg = torch.empty(self.ng, **f64)
        self._j_cg = torch.empty((self.nc, 3), **f64)
        self._p_cg = torch.empty(self.nc, **f64)
        self.a_gc = torch.empty((self.ng, 3), **f64)
        self._j_gc = torch.empty((self.ng, 3), **f64)
        self._p_gc = torch.empty(self.ng, **f64)
        if self.ng:
            self._galaxy_forces()
        self.block_steps = 0
        self._cross_valid = False   # a_cg, a_gc belong to the current positions

    # ---- pieces of the split ----------------------------------------------
    def _galaxy_forces(self):
        if self.cross == "tree":
            self._xgc[self.ng:] = self.cluster.pos
            self.ctx_g.tree_forces(self._xgc, self._mgc, self.eps2_g, self.theta, self.n_crit, self.g_frac,
                                   self._agc, self._pgc)
            self._tree_cg_valid = True
        elif self.field == "tree":
            self.ctx_g.tree_forces(self.xg, self.mg, self.eps2_g, self.theta, self.n_crit, self.g_frac, self.ag,
                                   self._pg)
        else:
            self.ctx_g.forces(self.xg, self.vg, self.mg, self.idx_g, self.eps2_g, self.ag, self._jg, self._pg)

    def cross_field(self):
        """Field of g on every particle of c and of c on every particle of g."""
        c = self.cluster
        if self.ng and self.nc:
            if self.cross == "tree":
                if not self._tree_cg_valid:
                    self._galaxy_forces()
            else:
                self.ctx_x.forces_ij(self.xg, self.vg, self.mg, c.pos, c.vel, self.idx_c, self.eps2_gc,
                                     self.a_cg, self._j_cg, self._p_cg)
            self.ctx_x.forces_ij(c.pos, c.vel, c.mass, self.xg, self.vg, self.idx_g, self.eps2_gc,
                                 self.a_gc, self._j_gc, self._p_gc)
        else:
            self.a_cg.zero_()
            self.a_gc.zero_()

    def kick(self, h):
        """e^{h A}: velocities of both subsystems move in the other's field
        (computed at the current positions unless a kick already did)."""
        if not self._cross_valid:
            self.cross_field()
            self._cross_valid = True
        self.ctx_x.kick(self.cluster.vel, self.a_cg, h)
        self.ctx_x.kick(self.vg, self.a_gc, h)

    def invalidate(self):
        """Forget the stored cross field (call after moving positions by hand)."""
        self._cross_valid = False
        self._tree_cg_valid = False

    def drift_cluster(self, use_graph=True):
        self._cross_valid = False
        self._tree_cg_valid = False
        c = self.cluster
        before = c.steps
        c.restart()
        c.run_to_tick((self.steps + 1) << c.max_level, use_graph=use_graph)
        self.block_steps += c.steps - before

    def drift_galaxy(self):
        self._cross_valid = False
        h = self.dt / self.n_sub
        for _ in range(self.n_sub):
            self.ctx_g.kick_drift(self.xg, self.vg, self.ag, 0.5 * h, h)
            self._galaxy_forces()
            self.ctx_g.kick(self.vg, self.ag, 0.5 * h)

    def step(self, use_graph=True):
        """One bridge step: half kick, both drifts, half kick."""
        self.kick(0.5 * self.dt)
        self.drift_cluster(use_graph)
        if self.ng:
            self.drift_galaxy()
        self.kick(0.5 * self.dt)
        self.steps += 1
        return self

    def run(self, n_steps, use_graph=True):
        for _ in range(n_steps):
            self.step(use_graph)
        return self

    @property
    def time(self):
        return self.steps * self.dt

    # ---- diagnostics ------------------------------------------------------
    def energy(self):
        """K_g + W_g + K_c + W_c + W_gc, each potential with its own softening."""
        c = self.cluster
        dev = c.dev
        out = torch.zeros(8, dtype=torch.float64, device=dev)
        parts = {}
        if self.ng:
            pot = torch.empty(self.ng, dtype=torch.float64, device=dev)
            self.ctx_g.forces(self.xg, self.vg, self.mg, self.idx_g, self.eps2_g, None, None, pot)   # W_g exactly
            o = self.ctx_g.energy(self.xg, self.vg, self.mg, pot, out).cpu().tolist()
            parts["Kg"], parts["Wg"] = o[0], o[1]
        else:
            parts["Kg"] = parts["Wg"] = 0.0
        pot = torch.empty(self.nc, dtype=torch.float64, device=dev)
        self.ctx_c.forces(c.pos, c.vel, c.mass, self.idx_c, self.eps2_c, None, None, pot)
        o = self.ctx_c.energy(c.pos, c.vel, c.mass, pot, out.zero_()).cpu().tolist()
        parts["Kc"], parts["Wc"] = o[0], o[1]
        if self.ng:
            pot = torch.empty(self.nc, dtype=torch.float64, device=dev)
            self.ctx_x.forces_ij(self.xg, self.vg, self.mg, c.pos, c.vel, self.idx_c, self.eps2_gc, None, None, pot)
            o = self.ctx_x.energy(c.pos, c.vel, c.mass, pot, out.zero_()).cpu().tolist()
            parts["Wgc"] = 2.0 * o[1]     # nb_energy halves the pair sum
        else:
            parts["Wgc"] = 0.0
        parts["E"] = parts["Kg"] + parts["Wg"] + parts["Kc"] + parts["Wc"] + parts["Wgc"]
        return parts
