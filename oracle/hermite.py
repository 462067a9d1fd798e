"""4th-order Hermite block-time-step integrator -- TEST INFRASTRUCTURE ONLY.

The paper names the integrator that the direct forces drive -- a fourth-order
Hermite predictor-corrector with individual block time steps (sections
"Simulating Collisional systems with direct force evaluation methods" and
"Simulating galaxy mergers with supermassive black holes") -- but writes none
of its formulas down.  This module follows the standard reading of that
scheme (Makino & Aarseth 1992), step by step, in plain numpy double
precision:

  predict    x_p = x + v d + a d^2/2 + j d^3/6,  v_p = v + a d + j d^2/2
  interpolate a2 = [-6(a0-a1) - dt(4 j0 + 2 j1)] / dt^2
              a3 = [12(a0-a1) + 6 dt (j0 + j1)] / dt^3
  correct    x1 = x_p + a2 dt^4/24 + a3 dt^5/120,  v1 = v_p + a2 dt^3/6 + a3 dt^4/24
  new step   dt* = sqrt(eta (|a1||a2e| + |j1|^2) / (|j1||a3| + |a2e|^2)),
             a2e = a2 + a3 dt  (the second derivative at the end of the step);
             a zero denominator gives dt* = dt_max
  levels     dt = dt_max 2^-level; if dt* < dt halve until dt <= dt*;
             else if dt* >= 2 dt, level > 0 and the new time is a multiple
             of 2 dt, double once; levels beyond max_level are clamped to it
             (and counted)
  startup    level = smallest k >= 0 with dt_max 2^-k <= eta |a|/|j|
  schedule   time in integer ticks of dt_max 2^-max_level;
             t_next = min_i (t_i + dt_i); active = {i : t_i + dt_i = t_next},
             ascending

The force routine is passed in (the oracle's ``forces_f64``/``forces_ld`` or a
closed-form field in the tests).
"""
from dataclasses import dataclass, field

import numpy as np


def predict(x, v, a, j, d):
    """Taylor predictor to offset d (scalar or per-row array)."""
    d = np.asarray(d, dtype=np.float64)
    if d.ndim == 1:
        d = d[:, None]
    xp = x + v * d + a * (d * d / 2.0) + j * (d * d * d / 6.0)
    vp = v + a * d + j * (d * d / 2.0)
    return xp, vp


def interpolate(a0, j0, a1, j1, dt):
    """Second and third derivative of a at the start of the step."""
    dt = np.asarray(dt, dtype=np.float64)
    if dt.ndim == 1:
        dt = dt[:, None]
    a2 = (-6.0 * (a0 - a1) - dt * (4.0 * j0 + 2.0 * j1)) / (dt * dt)
    a3 = (12.0 * (a0 - a1) + 6.0 * dt * (j0 + j1)) / (dt * dt * dt)
    return a2, a3


def correct(xp, vp, a2, a3, dt):
    dt = np.asarray(dt, dtype=np.float64)
    if dt.ndim == 1:
        dt = dt[:, None]
    x1 = xp + a2 * dt ** 4 / 24.0 + a3 * dt ** 5 / 120.0
    v1 = vp + a2 * dt ** 3 / 6.0 + a3 * dt ** 4 / 24.0
    return x1, v1


def _norm(u):
    return np.sqrt((u * u).sum(axis=-1))


def aarseth_dt(a1, j1, a2, a3, dt, eta, dt_max):
    """Aarseth's criterion evaluated at the end of the step."""
    dt = np.asarray(dt, dtype=np.float64)
    a2e = a2 + a3 * (dt[:, None] if dt.ndim == 1 else dt)
    num = _norm(a1) * _norm(a2e) + _norm(j1) ** 2
    den = _norm(j1) * _norm(a3) + _norm(a2e) ** 2
    out = np.full(np.shape(num), float(dt_max))
    ok = den > 0
    out[ok] = np.sqrt(eta * num[ok] / den[ok])
    return out


def new_level(level, dt_star, t_new, dt_max, max_level):
    """Power-of-two step levels.  Returns (new_level, clamped_mask)."""
    level = np.array(level, dtype=np.int64)
    out = level.copy()
    clamped = np.zeros(level.shape, dtype=bool)
    for n in range(level.size):
        L = int(level.flat[n])
        ds = float(np.asarray(dt_star).flat[n])
        dt = dt_max * 2.0 ** -L
        if ds < dt:
            while dt > ds and L < max_level:
                L += 1
                dt = dt_max * 2.0 ** -L
            clamped.flat[n] = dt > ds
        elif ds >= 2.0 * dt and L > 0:
            two_dt_ticks = 1 << (max_level - L + 1)
            if int(np.asarray(t_new).flat[n]) % two_dt_ticks == 0:
                L -= 1
        out.flat[n] = L
    return out, clamped


def startup_level(a, j, eta, dt_max, max_level):
    na, nj = _norm(a), _norm(j)
    lev = np.zeros(na.shape, dtype=np.int64)
    clamped = np.zeros(na.shape, dtype=bool)
    for n in range(na.size):
        if nj[n] == 0:
            continue
        target = eta * na[n] / nj[n]
        L = 0
        while dt_max * 2.0 ** -L > target and L < max_level:
            L += 1
        clamped[n] = dt_max * 2.0 ** -L > target
        lev[n] = L
    return lev, clamped


def energy(pos, vel, mass, pot):
    """K, W = 1/2 sum m phi, momentum P, angular momentum L."""
    K = 0.5 * float((mass * (vel * vel).sum(1)).sum())
    W = 0.5 * float((mass * pot).sum())
    P = (mass[:, None] * vel).sum(0)
    L = (mass[:, None] * np.cross(pos, vel)).sum(0)
    return dict(K=K, W=W, E=K + W, P=P, L=L)


@dataclass
class BlockState:
    x: np.ndarray
    v: np.ndarray
    m: np.ndarray
    a: np.ndarray
    j: np.ndarray
    t: np.ndarray          # int64 ticks
    level: np.ndarray      # int64
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


def initialise(x, v, m, eps2, eta, dt_max, max_level, forces):
    """All particles at t = 0: evaluate a, j and choose the startup levels."""
    n = m.shape[0]
    act = np.arange(n, dtype=np.int32)
    a, j, _ = forces(x, v, m, act)
    lev, cl = startup_level(a, j, eta, dt_max, max_level)
    return BlockState(x.copy(), v.copy(), m.copy(), a, j, np.zeros(n, dtype=np.int64), lev,
                      float(eps2), float(eta), float(dt_max), int(max_level),
                      force_evals=n, clamps=int(cl.sum()))


def block_step(st: BlockState, forces):
    """One block step: schedule, predict all, force on the active set, correct."""
    dt_ticks = np.left_shift(np.int64(1), (st.max_level - st.level).astype(np.int64))
    t_end = st.t + dt_ticks
    t_next = int(t_end.min())
    act = np.nonzero(t_end == t_next)[0].astype(np.int32)
    d_all = (t_next - st.t).astype(np.float64) * st.tick
    xp, vp = predict(st.x, st.v, st.a, st.j, d_all)
    a1, j1, _ = forces(xp, vp, st.m, act)
    dt = d_all[act]
    a2, a3 = interpolate(st.a[act], st.j[act], a1, j1, dt)
    x1, v1 = correct(xp[act], vp[act], a2, a3, dt)
    ds = aarseth_dt(a1, j1, a2, a3, dt, st.eta, st.dt_max)
    lev, cl = new_level(st.level[act], ds, np.full(act.size, t_next), st.dt_max, st.max_level)
    st.x[act], st.v[act], st.a[act], st.j[act] = x1, v1, a1, j1
    st.t[act] = t_next
    st.level[act] = lev
    st.steps += 1
    st.force_evals += act.size
    st.clamps += int(cl.sum())
    st.n_active_hist.append(act.size)
    return t_next, act


def run_until(st: BlockState, t_end: float, forces, max_steps=10 ** 9):
    """Block steps until every particle reaches t_end (a multiple of dt_max)."""
    end_ticks = int(round(t_end / st.tick))
    if end_ticks * st.tick != t_end:
        raise ValueError("t_end must be a whole number of ticks")
    while int(st.t.min()) < end_ticks:
        if st.steps >= max_steps:
            raise RuntimeError("step limit reached")
        block_step(st, forces)
    return st


def shared_step(x, v, a, j, m, dt, forces):
    """One shared-time-step Hermite step of every particle (for the Kepler pin)."""
    n = m.shape[0]
    xp, vp = predict(x, v, a, j, dt)
    a1, j1, _ = forces(xp, vp, m, np.arange(n, dtype=np.int32))
    a2, a3 = interpolate(a, j, a1, j1, dt)
    x1, v1 = correct(xp, vp, a2, a3, dt)
    return x1, v1, a1, j1
