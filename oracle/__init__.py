"""CPU oracle for the direct-summation N-body hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never does,
and the two share no code: the only shared module is ``synth`` (seeded input
generators, which hold none of the method's arithmetic).

Contents
  forces_f64 / forces_ld   plain O(N^2) sums (C, ``forces.c``)
  pair_potential_energy    W as a sum over pairs i<j (C)
  snap_ld                  acceleration, jerk, snap and potential (C, ``snap.c``)
  hermite                  4th-order Hermite block-step integrator (numpy)
  hermite6                 6th-order Hermite block-step integrator (numpy)
  bridge                   kick-drift-kick split of two subsystems (numpy)
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        # NB_ORACLE_LIB lets the mutation tests load a deliberately broken build
        path = os.environ.get("NB_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_forces_f64.restype = ctypes.c_int64
        lib.oracle_forces_f64.argtypes = [dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                          ctypes.c_double, dp, dp, dp, ctypes.c_int]
        lib.oracle_forces_ld.restype = ctypes.c_int64
        lib.oracle_forces_ld.argtypes = [dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64,
                                         ctypes.c_double, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_pair_potential_energy.restype = ctypes.c_double
        lib.oracle_pair_potential_energy.argtypes = [dp, dp, ctypes.c_int64, ctypes.c_double]
        _LIB = lib
    return _LIB


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(pos, vel, mass, active):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    n = mass.shape[0]
    if pos.shape != (n, 3) or vel.shape != (n, 3):
        raise ValueError("pos/vel must be (N,3) and mass (N,)")
    if active is None:
        active = np.arange(n, dtype=np.int32)
    active = np.ascontiguousarray(active, dtype=np.int32)
    if active.size and (active.min() < 0 or active.max() >= n):
        raise ValueError("active index out of range")
    return pos, vel, mass, active


def forces_f64(pos, vel, mass, eps2, active=None, nthreads=0):
    """Acceleration, jerk, potential in plain IEEE double (j ascending).

    Returns (acc [n_active,3], jerk [n_active,3], pot [n_active], skipped)."""
    pos, vel, mass, active = _prep(pos, vel, mass, active)
    na = active.shape[0]
    acc = np.zeros((na, 3)); jerk = np.zeros((na, 3)); pot = np.zeros(na)
    sk = _lib().oracle_forces_f64(_d(pos), _d(vel), _d(mass), mass.shape[0],
                                  active.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), na,
                                  float(eps2), _d(acc), _d(jerk), _d(pot), int(nthreads))
    return acc, jerk, pot, int(sk)


def forces_ld(pos, vel, mass, eps2, active=None, nthreads=0):
    """Same sums in x87 extended precision, rounded to double at the end.

    Returns a dict with acc, jerk, pot and the per-row magnitude sums
    abs_acc = sum_j |a_ij|, abs_jerk = sum_j |jdot_ij|, abs_pot = sum_j m_j/s^1/2,
    plus the count of skipped coincident pairs."""
    pos, vel, mass, active = _prep(pos, vel, mass, active)
    na = active.shape[0]
    acc = np.zeros((na, 3)); jerk = np.zeros((na, 3)); pot = np.zeros(na)
    aa = np.zeros(na); aj = np.zeros(na); ap = np.zeros(na)
    sk = _lib().oracle_forces_ld(_d(pos), _d(vel), _d(mass), mass.shape[0],
                                 active.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), na,
                                 float(eps2), _d(acc), _d(jerk), _d(pot), _d(aa), _d(aj), _d(ap),
                                 int(nthreads))
    return dict(acc=acc, jerk=jerk, pot=pot, abs_acc=aa, abs_jerk=aj, abs_pot=ap, skipped=int(sk))


def pair_potential_energy(pos, mass, eps2):
    """W = -sum_{i<j} m_i m_j / sqrt(r_ij^2 + eps2) (extended precision)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    return float(_lib().oracle_pair_potential_energy(_d(pos), _d(mass), mass.shape[0], float(eps2)))


_SNAP = None


def _snap_lib():
    global _SNAP
    if _SNAP is None:
        # NB_ORACLE_SNAP_LIB lets the mutation tests load a deliberately broken build
        path = os.environ.get("NB_ORACLE_SNAP_LIB") or os.path.join(_HERE, "liboracle_snap.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_snap_ld.restype = ctypes.c_int64
        lib.oracle_snap_ld.argtypes = [dp, dp, dp, dp, ctypes.c_int64, ip, ctypes.c_int64, ctypes.c_double,
                                       dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        _SNAP = lib
    return _SNAP


def snap_ld(pos, vel, acc_j, mass, eps2, active=None, nthreads=0):
    """Acceleration, jerk, snap and potential in extended precision, each
    particle moving with its own acceleration ``acc_j`` [N,3] at the instant.

    Returns a dict with acc, jerk, snap, pot, the magnitude sums abs_acc,
    abs_jerk, abs_snap, abs_pot and the count of skipped coincident pairs."""
    pos, vel, mass, active = _prep(pos, vel, mass, active)
    acc_j = np.ascontiguousarray(acc_j, dtype=np.float64)
    if acc_j.shape != pos.shape:
        raise ValueError("acc_j must be (N,3)")
    na = active.shape[0]
    out = {k: np.zeros((na, 3)) for k in ("acc", "jerk", "snap")}
    out["pot"] = np.zeros(na)
    ab = {k: np.zeros(na) for k in ("abs_acc", "abs_jerk", "abs_snap", "abs_pot")}
    sk = _snap_lib().oracle_snap_ld(_d(pos), _d(vel), _d(acc_j), _d(mass), mass.shape[0],
                                    active.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), na, float(eps2),
                                    _d(out["acc"]), _d(out["jerk"]), _d(out["snap"]), _d(out["pot"]),
                                    _d(ab["abs_acc"]), _d(ab["abs_jerk"]), _d(ab["abs_snap"]), _d(ab["abs_pot"]),
                                    int(nthreads))
    out.update(ab)
    out["skipped"] = int(sk)
    return out
