"""6th-order Hermite block-time-step integrator -- TEST INFRASTRUCTURE ONLY.

The paper cites Hermite schemes of order higher than four for the direct
method (section "Simulating Collisional systems with direct force evaluation
methods") and writes none of them down.  This module is the reading the
library implements, written out in plain numpy double precision, step by
step:

  forces     acceleration a, jerk j and snap s of every active particle, each
             particle moving with its own predicted x, v and a (oracle.snap_ld)
  predict    x_p = x + v d + a d^2/2 + j d^3/6 + s d^4/24 + c d^5/120
             v_p = v + a d + j d^2/2 + s d^3/6 + c d^4/24
             a_p = a + j d + s d^2/2 + c d^3/6
             (c the crackle kept from the particle's last step; 0 at start)
  interpolate the quintic a(t) = a0 + j0 t + s0 t^2/2 + c0 t^3/6 + p0 t^4/24
             + q0 t^5/120 through (a0, j0, s0) at t = 0 and (a1, j1, s1) at
             t = dt: c0, p0, q0 solve that 3x3 linear system (per component)
  correct    x1, v1 = the exact integral of that quintic:
             v1 = v0 + a0 dt + j0 dt^2/2 + s0 dt^3/6 + c0 dt^4/24 + p0 dt^5/120 + q0 dt^6/720
             x1 = x0 + v0 dt + a0 dt^2/2 + j0 dt^3/6 + s0 dt^4/24 + c0 dt^5/120
                  + p0 dt^6/720 + q0 dt^7/5040
             and the end-of-step derivatives c1 = c0 + p0 dt + q0 dt^2/2,
             p1 = p0 + q0 dt
  new step   generalised Aarseth criterion of order six,
             dt* = eta ((sqrt(|a1||s1|) + |j1|) / (sqrt(|c1||q0|) + |p1|))^(1/3);
             a zero denominator gives dt_max
  levels     the power-of-two rules of oracle.hermite.new_level
  startup    a, j (pass 1), then s with every particle's a (pass 2), c = 0;
             dt* = eta_s min(|a|/|j|, sqrt(|a|/|s|)) over the finite terms
             (dt_max if none), level = smallest k >= 0 with dt_max 2^-k <= dt*
  schedule   as oracle.hermite (integer ticks, ascending active set)

The force routine is passed in: forces6(x, v, a, m, act) -> (a, j, s, pot).
"""
from dataclasses import dataclass, field

import numpy as np

from . import hermite as H


def predict(x, v, a, j, s, c, d):
    d = np.asarray(d, dtype=np.float64)
    if d.ndim == 1:
        d = d[:, None]
    xp = x + v * d + a * d ** 2 / 2.0 + j * d ** 3 / 6.0 + s * d ** 4 / 24.0 + c * d ** 5 / 120.0
    vp = v + a * d + j * d ** 2 / 2.0 + s * d ** 3 / 6.0 + c * d ** 4 / 24.0
    ap = a + j * d + s * d ** 2 / 2.0 + c * d ** 3 / 6.0
    return xp, vp, ap


def interpolate(a0, j0, s0, a1, j1, s1, dt):
    """Crackle, pop and the fifth derivative of a at the start of the step."""
    a0, j0, s0, a1, j1, s1 = (np.asarray(t, dtype=np.float64) for t in (a0, j0, s0, a1, j1, s1))
    n = a0.shape[0]
    dt = np.broadcast_to(np.asarray(dt, dtype=np.float64), (n,))
    out = np.empty((3, n, 3))
    for k in range(n):
        h = float(dt[k])
        # unknowns (c0, p0, q0); rows: a(h), a'(h), a''(h) minus the known part
        M = np.array([[h ** 3 / 6, h ** 4 / 24, h ** 5 / 120],
                      [h ** 2 / 2, h ** 3 / 6, h ** 4 / 24],
                      [h, h ** 2 / 2, h ** 3 / 6]])
        rhs = np.stack([a1[k] - (a0[k] + j0[k] * h + s0[k] * h * h / 2),
                        j1[k] - (j0[k] + s0[k] * h),
                        s1[k] - s0[k]])
        out[:, k, :] = np.linalg.solve(M, rhs)
    return out[0], out[1], out[2]


def correct(x0, v0, a0, j0, s0, c0, p0, q0, dt):
    dt = np.asarray(dt, dtype=np.float64)
    if dt.ndim == 1:
        dt = dt[:, None]
    v1 = v0 + a0 * dt + j0 * dt ** 2 / 2 + s0 * dt ** 3 / 6 + c0 * dt ** 4 / 24 + p0 * dt ** 5 / 120 \
        + q0 * dt ** 6 / 720
    x1 = x0 + v0 * dt + a0 * dt ** 2 / 2 + j0 * dt ** 3 / 6 + s0 * dt ** 4 / 24 + c0 * dt ** 5 / 120 \
        + p0 * dt ** 6 / 720 + q0 * dt ** 7 / 5040
    c1 = c0 + p0 * dt + q0 * dt ** 2 / 2
    p1 = p0 + q0 * dt
    return x1, v1, c1, p1


def _norm(u):
    return np.sqrt((u * u).sum(axis=-1))


def new_dt(a1, j1, s1, c1, p1, q, eta, dt_max):
    num = np.sqrt(_norm(a1) * _norm(s1)) + _norm(j1)
    den = np.sqrt(_norm(c1) * _norm(q)) + _norm(p1)
    out = np.full(np.shape(num), float(dt_max))
    ok = den > 0
    out[ok] = eta * (num[ok] / den[ok]) ** (1.0 / 3.0)
    return out


def startup_level(a, j, s, eta_s, dt_max, max_level):
    na, nj, ns = _norm(a), _norm(j), _norm(s)
    lev = np.zeros(na.shape, dtype=np.int64)
    clamped = np.zeros(na.shape, dtype=bool)
    for n in range(na.size):
        cand = []
        if nj[n] > 0:
            cand.append(na[n] / nj[n])
        if ns[n] > 0:
            cand.append(np.sqrt(na[n] / ns[n]))
        if not cand:
            continue
        target = eta_s * min(cand)
        L = 0
        while dt_max * 2.0 ** -L > target and L < max_level:
            L += 1
        clamped[n] = dt_max * 2.0 ** -L > target
        lev[n] = L
    return lev, clamped


@dataclass
class BlockState6:
    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    a: np.ndarray
    j: np.ndarray
    s: np.ndarray
    c: np.ndarray
    t: np.ndarray          # int64 ticks
    level: np.ndarray
    eps2: float
    eta: float
    dt_max: float
    max_level: int
    steps: int = 0
    force_evals: int = 0
    clamps: int = 0
    n_active_hist: list = field(default_factory=list)

    @property
    def tick(self):
        return self.dt_max * 2.0 ** -self.max_level


def initialise(x, v, m, eps2, eta, eta_s, dt_max, max_level, forces6):
    """All particles at t = 0: a and j, then s with those a; c = 0; start-up levels."""
    n = m.shape[0]
    act = np.arange(n, dtype=np.int32)
    a, j, _, _ = forces6(x, v, np.zeros_like(x), m, act)
    a, j, s, _ = forces6(x, v, a, m, act)
    lev, cl = startup_level(a, j, s, eta_s, dt_max, max_level)
    return BlockState6(x.copy(), v.copy(), m.copy(), a, j, s, np.zeros_like(a), np.zeros(n, dtype=np.int64), lev,
                       float(eps2), float(eta), float(dt_max), int(max_level), force_evals=2 * n,
                       clamps=int(cl.sum()))


def block_step(st: BlockState6, forces6):
    dt_ticks = np.left_shift(np.int64(1), (st.max_level - st.level).astype(np.int64))
    t_end = st.t + dt_ticks
    t_next = int(t_end.min())
    act = np.nonzero(t_end == t_next)[0].astype(np.int32)
    d_all = (t_next - st.t).astype(np.float64) * st.tick
    xp, vp, ap = predict(st.x, st.v, st.a, st.j, st.s, st.c, d_all)
    a1, j1, s1, _ = forces6(xp, vp, ap, st.m, act)
    dt = d_all[act]
    c0, p0, q0 = interpolate(st.a[act], st.j[act], st.s[act], a1, j1, s1, dt)
    x1, v1, c1, p1 = correct(st.x[act], st.v[act], st.a[act], st.j[act], st.s[act], c0, p0, q0, dt)
    ds = new_dt(a1, j1, s1, c1, p1, q0, st.eta, st.dt_max)
    lev, cl = H.new_level(st.level[act], ds, np.full(act.size, t_next), st.dt_max, st.max_level)
    st.x[act], st.v[act], st.a[act], st.j[act], st.s[act], st.c[act] = x1, v1, a1, j1, s1, c1
    st.t[act] = t_next
    st.level[act] = lev
    st.steps += 1
    st.force_evals += act.size
    st.clamps += int(cl.sum())
    st.n_active_hist.append(act.size)
    return t_next, act


def run_until(st: BlockState6, t_end: float, forces6, max_steps=10 ** 9):
    end_ticks = int(round(t_end / st.tick))
    if end_ticks * st.tick != t_end:
        raise ValueError("t_end must be a whole number of ticks")
    while int(st.t.min()) < end_ticks:
        if st.steps >= max_steps:
            raise RuntimeError("step limit reached")
        block_step(st, forces6)
    return st


def shared_step(x, v, a, j, s, c, m, dt, forces6):
    """One shared-time-step step of every particle (for the Kepler order pin)."""
    n = m.shape[0]
    xp, vp, ap = predict(x, v, a, j, s, c, dt)
    a1, j1, s1, _ = forces6(xp, vp, ap, m, np.arange(n, dtype=np.int32))
    dts = np.full(n, float(dt))
    c0, p0, q0 = interpolate(a, j, s, a1, j1, s1, dts)
    x1, v1, c1, _ = correct(x, v, a, j, s, c0, p0, q0, dts)
    return x1, v1, a1, j1, s1, c1


def oracle_forces6(eps2):
    """The oracle's force routine in the form this module expects."""
    from . import snap_ld

    def f(x, v, a, m, act):
        r = snap_ld(x, v, a, m, eps2, act)
        return r["acc"], r["jerk"], r["snap"], r["pot"]
    return f
