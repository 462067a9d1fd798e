"""Second-order Hamiltonian split ("bridge") of a collisional subsystem and
a field subsystem -- TEST INFRASTRUCTURE ONLY.

Section "The multi-scale approach" writes the Hamiltonian of the whole system
as H = H_A + H_B, where H_A = W_gc is the potential energy between the galaxy
particles (g) and the stars in the sphere of influence of the central black
holes (c), and H_B = (K_g + W_g) + (K_c + W_c) = H_g + H_c.  The evolution over
dt is taken to second order as e^{dt/2 A} e^{dt B} e^{dt/2 A} (A and B the
Poisson-bracket operators of H_A and H_B); e^{dt B} factors into separate
evolutions of g and c because H_B has no cross term.  Written out
(kick-drift-kick):

  kick(h)    every particle of c: v += h a_{c<-g}(x); every particle of g:
             v += h a_{g<-c}(x).  H_A depends on positions only, so the
             positions stay.
  drift(dt)  c advances under H_c alone with the block-step Hermite scheme
             (oracle.hermite).  The kick changed its velocities, so every
             drift restarts it: new a and jdot, start-up levels.  Its dt_max
             is the bridge step, so each drift ends on a synchronisation time.
             g advances under H_g alone with n_sub shared-step leapfrog
             substeps (kick-drift-kick) of h = dt/n_sub with its own forces
             (the paper's tree code, or a direct sum; the field solver is not
             part of the split).

The field subsystem's own forces come from a routine passed in (``field``:
positions and masses -> accelerations); by default the direct sum, or the
oracle's tree code through ``tree_field``.

Cross field (``cross``).  "direct": both directions are direct sums.  "tree":
each subsystem's own solver gives the field it exerts, as when the two codes
of the paper's hybrid are coupled -- the field of g on c comes from g's tree
code, evaluated together with g's own forces on the combined set [g | c] with
the masses of c set to zero (so c feels g and exerts nothing), and the field
of c on g is the direct sum over c.  It needs eps2_gc = eps2_g (one tree
evaluation serves both) and is taken at every evaluation of g's forces, which
the bridge step makes at the positions its closing kick uses.

Softening: eps2_g inside g, eps2_c inside c, eps2_gc across.  Arithmetic of
the elementwise updates, in this order and without fused multiply-adds:
v + (h/2) a, then x + h v.

The force sums are the oracle's own direct sums (``forces_f64``); the field
of g on the particles of c (and the reverse) is that sum over the
concatenated set [g | c] with the receiving subsystem's masses set to zero,
so only the other subsystem exerts (the i-set/j-set split of the paper's
section on GPU optimisations).
"""
from dataclasses import dataclass

import numpy as np

from . import forces_f64
from . import hermite


def cross_forces(x_i, v_i, x_j, v_j, m_j, eps2):
    """Acceleration, jerk and potential on every particle of i in the field of j.

    Returns (acc [Ni,3], jerk [Ni,3], pot [Ni])."""
    x_i, v_i = np.asarray(x_i, dtype=np.float64), np.asarray(v_i, dtype=np.float64)
    nj = np.asarray(m_j).shape[0]
    ni = x_i.shape[0]
    pos = np.concatenate([x_j, x_i])
    vel = np.concatenate([v_j, v_i])
    mass = np.concatenate([np.asarray(m_j, dtype=np.float64), np.zeros(ni)])
    act = np.arange(nj, nj + ni, dtype=np.int32)
    a, j, p, _ = forces_f64(pos, vel, mass, eps2, act)
    return a, j, p


def self_forces(eps2):
    """Force routine in the form oracle.hermite expects: (x, v, m, act) -> (a, j, pot)."""
    def f(x, v, m, act):
        a, j, p, _ = forces_f64(x, v, m, eps2, act)
        return a, j, p
    return f


def direct_field(eps2):
    """g's own accelerations by the direct sum."""
    def f(x, m):
        return self_forces(eps2)(x, np.zeros_like(x), m, np.arange(m.shape[0], dtype=np.int32))[0]
    return f


def tree_field(eps2, theta, n_crit=16, g_frac=1.0 / 16):
    """g's own accelerations by the oracle's tree code."""
    from . import tree as TR

    def f(x, m):
        t = TR.build(x, m, n_crit)
        return TR.forces(x, m, eps2, theta, n_crit, g_max=g_frac * t.side, tree=t)[0]
    return f


def galaxy_and_cross_tree(xg, mg, xc, eps2, theta, n_crit=16, g_frac=1.0 / 16):
    """One tree evaluation on [g | c] with c massless: (g's own acceleration,
    the acceleration of c in the field of g)."""
    from . import tree as TR
    ng = np.asarray(mg).shape[0]
    x = np.concatenate([np.asarray(xg, dtype=np.float64), np.asarray(xc, dtype=np.float64)])
    m = np.concatenate([np.asarray(mg, dtype=np.float64), np.zeros(np.asarray(xc).shape[0])])
    t = TR.build(x, m, n_crit)
    a = TR.forces(x, m, eps2, theta, n_crit, g_max=g_frac * t.side, tree=t)[0]
    return a[:ng], a[ng:]


@dataclass
class BridgeState:
    xg: np.ndarray
    vg: np.ndarray
    mg: np.ndarray
    ag: np.ndarray                 # self acceleration of g at xg
    cluster: hermite.BlockState    # c, with dt_max = the bridge step
    eps2_g: float
    eps2_c: float
    eps2_gc: float
    dt: float
    n_sub: int
    field: object = None
    steps: int = 0
    cross: str = "direct"
    tree_args: tuple = ()          # (theta, n_crit, g_frac) for cross = "tree"
    a_cg: np.ndarray = None        # field of g on c from g's tree (cross = "tree")

    @property
    def time(self):
        return self.steps * self.dt


def initialise(xg, vg, mg, xc, vc, mc, eps2_g, eps2_c, eps2_gc, dt, n_sub=1, eta=0.01, max_level=30, field=None,
               cross="direct", theta=0.5, n_crit=16, g_frac=1.0 / 16):
    xg = np.array(xg, dtype=np.float64)
    vg = np.array(vg, dtype=np.float64)
    mg = np.array(mg, dtype=np.float64)
    if cross not in ("direct", "tree"):
        raise ValueError("cross must be 'direct' or 'tree'")
    if cross == "tree" and eps2_gc != eps2_g:
        raise ValueError("cross = 'tree' needs eps2_gc == eps2_g")
    field = field if field is not None else direct_field(eps2_g)
    cl = hermite.initialise(np.asarray(xc, dtype=np.float64), np.asarray(vc, dtype=np.float64),
                            np.asarray(mc, dtype=np.float64), eps2_c, eta, dt, max_level, self_forces(eps2_c))
    st = BridgeState(xg, vg, mg, np.zeros((0, 3)), cl, float(eps2_g), float(eps2_c), float(eps2_gc), float(dt),
                     int(n_sub), field, cross=cross, tree_args=(float(theta), int(n_crit), float(g_frac)))
    st.a_cg = np.zeros_like(cl.x)
    if mg.shape[0]:
        galaxy_forces(st)
    return st


def galaxy_forces(st: BridgeState):
    """g's own accelerations at the current positions (and, with cross = "tree",
    the field of g on c from the same tree evaluation)."""
    if st.cross == "tree":
        st.ag, st.a_cg = galaxy_and_cross_tree(st.xg, st.mg, st.cluster.x, st.eps2_g, *st.tree_args)
    else:
        st.ag = st.field(st.xg, st.mg)


def kick(st: BridgeState, h):
    """e^{h A}: both subsystems take the other's field at the current positions."""
    c = st.cluster
    if st.cross == "tree":
        a_cg = st.a_cg
    else:
        a_cg = cross_forces(c.x, c.v, st.xg, st.vg, st.mg, st.eps2_gc)[0]
    a_gc = cross_forces(st.xg, st.vg, c.x, c.v, c.m, st.eps2_gc)[0]
    c.v = c.v + h * a_cg
    st.vg = st.vg + h * a_gc


def drift_cluster(st: BridgeState):
    """c under H_c for one bridge step: restart, then block steps to the next synchronisation time."""
    c = st.cluster
    n = c.m.shape[0]
    c.a, c.j, _ = self_forces(st.eps2_c)(c.x, c.v, c.m, np.arange(n, dtype=np.int32))
    lev, cl = hermite.startup_level(c.a, c.j, c.eta, c.dt_max, c.max_level)
    c.level = lev
    c.clamps += int(cl.sum())
    c.force_evals += n
    hermite.run_until(c, (st.steps + 1) * st.dt, self_forces(st.eps2_c))


def drift_galaxy(st: BridgeState):
    """g under H_g for one bridge step: n_sub leapfrog substeps (kick-drift-kick)."""
    h = st.dt / st.n_sub
    for _ in range(st.n_sub):
        st.vg = st.vg + (0.5 * h) * st.ag
        st.xg = st.xg + h * st.vg
        galaxy_forces(st)
        st.vg = st.vg + (0.5 * h) * st.ag


def step(st: BridgeState):
    """One bridge step: half kick, both drifts, half kick."""
    kick(st, 0.5 * st.dt)
    drift_cluster(st)
    if st.mg.shape[0]:
        drift_galaxy(st)
    kick(st, 0.5 * st.dt)
    st.steps += 1
    return st


def energy(st: BridgeState):
    """K_g + W_g + K_c + W_c + W_gc, each potential with its own softening."""
    c = st.cluster
    ng, nc = st.mg.shape[0], c.m.shape[0]
    Kg = 0.5 * float((st.mg * (st.vg * st.vg).sum(1)).sum())
    Kc = 0.5 * float((c.m * (c.v * c.v).sum(1)).sum())
    Wg = 0.5 * float((st.mg * self_forces(st.eps2_g)(st.xg, st.vg, st.mg, np.arange(ng, dtype=np.int32))[2]).sum())
    Wc = 0.5 * float((c.m * self_forces(st.eps2_c)(c.x, c.v, c.m, np.arange(nc, dtype=np.int32))[2]).sum())
    Wgc = float((c.m * cross_forces(c.x, c.v, st.xg, st.vg, st.mg, st.eps2_gc)[2]).sum())
    return dict(Kg=Kg, Wg=Wg, Kc=Kc, Wc=Wc, Wgc=Wgc, E=Kg + Wg + Kc + Wc + Wgc)
