"""Python binding of the MI355X direct-summation N-body library.

A thin ctypes layer over ``libnbody.so`` (the C ABI in ``include/nbody.h``):
argument marshalling only -- every step of the computation runs in the HIP
kernels.  PyTorch provides device memory and streams; arrays are torch
tensors on the context's GPU (float64 (n,3) / (n,) contiguous, int32 index
arrays, int64 tick arrays).

If the shared library has not been built this module raises ImportError:
there is no CPU fallback.
"""
import ctypes
import os
import sys

import torch

__all__ = ["NbodyError", "Context", "PREC_FP64", "PREC_MIXED", "PREC_MIXED_DS", "lib_path", "library",
           "nbody_forces", "nbody_forces_noalloc", "nbody_forces_devcount", "nbody_forces_batch", "hermite_predict",
           "hermite_correct", "hermite_startup", "nb_schedule", "nb_block_step", "nb_energy",
           "nbody_forces_ij", "nb_kick", "nb_kick_drift", "nbody_forces6", "hermite6_predict",
           "hermite6_correct", "hermite6_startup", "nb_block_step6", "nb_tree_forces", "nb_sync",
           "check_active_host"]

PREC_FP64 = 0
PREC_MIXED = 1
PREC_MIXED_DS = 2
_PREC_NAMES = {"fp64": PREC_FP64, "f64": PREC_FP64, "mixed": PREC_MIXED, "mixed_ds": PREC_MIXED_DS}

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libnbody.so")

if not os.path.exists(lib_path):
    raise ImportError(f"{lib_path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(lib_path)


def _log_level():
    """NB_LOG as an integer (0 when unset, empty or not a number); the
    library reads the same variable when a context is created."""
    try:
        return max(0, int(os.environ.get("NB_LOG", "") or 0))
    except ValueError:
        return 0

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_int = ctypes.c_int


def _sig(name, *args):
    f = getattr(_lib, name)
    f.restype = _int
    f.argtypes = list(args)
    return f


_lib.nb_version.restype = ctypes.c_char_p
_lib.nb_version.argtypes = []
_lib.nb_last_error.restype = ctypes.c_char_p
_lib.nb_last_error.argtypes = [_vp]
_sig("nb_create", ctypes.POINTER(_vp), _int, _int)
_sig("nb_destroy", _vp)
_sig("nb_set_stream", _vp, _vp)
_sig("nb_set_precision", _vp, _int)
_sig("nb_workspace_bytes", _vp, ctypes.POINTER(_i64))
_lib.nb_get_precision.restype = _int
_lib.nb_get_precision.argtypes = [_vp]
_sig("nb_set_launch", _vp, _int, _int, _int, _int, _int)
_sig("nb_get_launch", _vp, _i64, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int), ctypes.POINTER(_int),
     ctypes.POINTER(_int), ctypes.POINTER(_int))
_sig("nb_tune_add", _vp, _int, _i64, _i64, _i64, _int, _int, _int, _int, _int)
_sig("nb_tune_add_batch", _vp, _int, _int, _i64, _i64, _int, _int)
_sig("nb_set_split_sum", _vp, _int)
_sig("nb_get_batch_launch", _vp, _int, _i64, _i64, ctypes.POINTER(_int), ctypes.POINTER(_int))
_sig("nb_tune_clear", _vp)
_sig("nb_set_stop_source", _vp, _vp)
_sig("nb_set_phase_timing", _vp, _int)
_sig("nb_phase_times", _vp, ctypes.POINTER(ctypes.c_float))
_sig("nb_time_forces", _vp, _int, _int, _int, _int, _int, _vp, _vp, _vp, _i64, _vp, _i64, _dbl, _vp, _vp, _vp, _int,
     ctypes.POINTER(_dbl))
_sig("nbody_forces", _vp, _vp, _vp, _vp, _i64, _vp, _i64, _dbl, _vp, _vp, _vp)
_sig("nbody_forces_noalloc", _vp, _vp, _vp, _vp, _i64, _vp, _i64, _dbl, _vp, _vp, _vp)
_sig("nbody_forces_devcount", _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _dbl, _vp, _vp, _vp)
_sig("nbody_forces_ij", _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _dbl, _vp, _vp, _vp)
_sig("nbody_forces6", _vp, _vp, _vp, _vp, _vp, _i64, _vp, _i64, _dbl, _vp, _vp, _vp, _vp)
_sig("hermite6_predict", _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _dbl, _i64, _vp, _vp, _vp)
_sig("hermite6_correct", _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl,
     _i32, _vp)
_sig("hermite6_startup", _vp, _vp, _vp, _vp, _i64, _dbl, _dbl, _i32, _vp)
_sig("nb_block_step6", _vp, _i64, _dbl, _dbl, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64)
_sig("nb_tree_forces", _vp, _vp, _vp, _i64, _dbl, _dbl, _i32, _dbl, _vp, _vp, _vp)
_sig("nb_tree_keys", _vp, _vp, _i64, _vp, _vp)
_sig("nb_kick", _vp, _vp, _vp, _i64, _dbl)
_sig("nb_kick_drift", _vp, _vp, _vp, _vp, _i64, _dbl, _dbl)
_sig("hermite_predict", _vp, _vp, _vp, _vp, _vp, _vp, _i64, _dbl, _i64, _vp, _vp)
_sig("hermite_correct", _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _dbl, _i32,
     _vp)
_sig("nb_sync", _vp)
_sig("nb_check_active_host", _vp, _i64, _i64, _i64, ctypes.POINTER(_i64))
_sig("hermite_startup", _vp, _vp, _vp, _i64, _dbl, _dbl, _i32, _vp)
_sig("nb_schedule", _vp, _vp, _vp, _i64, _i32, _vp, _vp)
_sig("nb_block_step", _vp, _i64, _dbl, _dbl, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
     _vp, _vp, _vp, _vp, _i64)
_sig("nb_energy", _vp, _vp, _vp, _vp, _vp, _i64, _vp)
_sig("nbody_forces_batch", _vp, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp)
_sig("nb_block_step_batch", _vp, _vp, _i64, _vp, _dbl, _dbl, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
     _vp, _vp, _vp, _vp, _vp, _i64)


def check_active_host(active, lo, hi):
    """Index of the first entry of the host int32 array ``active`` outside
    [lo, hi), or -1 (``nb_check_active_host``; no device needed)."""
    import numpy as np
    a = np.ascontiguousarray(active, dtype=np.int32)
    bad = _i64()
    rc = _lib.nb_check_active_host(a.ctypes.data_as(_vp), a.shape[0], int(lo), int(hi), ctypes.byref(bad))
    if rc not in (0, -1):
        raise NbodyError(rc, "nb_check_active_host")
    return bad.value


def library():
    """The loaded ctypes library (for tests that check the exported symbols)."""
    return _lib


class NbodyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nbody error {code}: {msg}")
        self.code = code


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_vec(t, n, name, dev):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device != dev:
        raise TypeError(f"{name}: float64 tensor on {dev} required")
    if t.shape != (n, 3) or not t.is_contiguous():
        raise ValueError(f"{name}: contiguous ({n}, 3) required, got {tuple(t.shape)}")


def _check_1d(t, n, name, dtype, dev):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != dev:
        raise TypeError(f"{name}: {dtype} tensor on {dev} required")
    if t.shape != (n,) or not t.is_contiguous():
        raise ValueError(f"{name}: contiguous ({n},) required, got {tuple(t.shape)}")


class Context:
    """One library context on one GPU (``nb_create``)."""

    def __init__(self, device=0, precision="fp64", stream=None, load_tuning=True):
        """load_tuning: install a saved launch table -- the file named by the
        environment variable NB_TUNE_CACHE when set, else the autotuner's
        table for this GPU (``tuning_gfx950.json`` next to this file) when it
        exists (``autotune.table_path``)."""
        prec = _PREC_NAMES[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        rc = _lib.nb_create(ctypes.byref(h), int(device), prec)
        if rc != 0:
            raise NbodyError(rc, "nb_create failed (no usable gfx950 device?)")
        self._h = h
        self.device = torch.device("cuda", int(device))
        self.set_stream(stream)
        self.tuning_table = None
        if load_tuning:
            from . import autotune
            path = autotune.table_path()
            if path:
                n = autotune.load(self, path)
                self.tuning_table = path
                if _log_level() >= 2:
                    print(f"nbody: launch table {path} ({n} entries)", file=sys.stderr, flush=True)

    def _chk(self, rc):
        if rc != 0:
            raise NbodyError(rc, _lib.nb_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.nb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def sync(self):
        """Wait for the context's stream; raise NbodyError (NB_EINVAL) if a
        kernel met an active_idx entry outside its valid range since the last
        sync (``nb_sync``)."""
        self._chk(_lib.nb_sync(self._h))

    def workspace_bytes(self):
        """Device bytes held by the growable workspace and mirror (``nb_workspace_bytes``)."""
        b = _i64()
        self._chk(_lib.nb_workspace_bytes(self._h, ctypes.byref(b)))
        return b.value

    @property
    def stream(self):
        """The torch.cuda.Stream the context launches on."""
        return self._stream

    def set_stream(self, stream=None):
        """Launch on ``stream`` (a torch.cuda.Stream), default torch's current stream."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = s
        self._chk(_lib.nb_set_stream(self._h, ctypes.c_void_p(s.cuda_stream)))

    @property
    def precision(self):
        return _lib.nb_get_precision(self._h)

    def set_precision(self, precision):
        prec = _PREC_NAMES[precision] if isinstance(precision, str) else int(precision)
        self._chk(_lib.nb_set_precision(self._h, prec))

    def set_launch(self, K=0, L=1, S=0, T=0, WG=0):
        """Force (K, L, S) and the tile T / workgroup size WG (0: 256); K = 0 restores automatic choice."""
        self._chk(_lib.nb_set_launch(self._h, int(K), int(L), int(S), int(T), int(WG)))

    def get_shape(self, N, n_active):
        """(K, L, S, T, WG) of the launch the context would use."""
        K, L, S, T, WG = _int(), _int(), _int(), _int(), _int()
        self._chk(_lib.nb_get_launch(self._h, int(N), int(n_active), ctypes.byref(K), ctypes.byref(L),
                                     ctypes.byref(S), ctypes.byref(T), ctypes.byref(WG)))
        return K.value, L.value, S.value, T.value, WG.value

    def get_launch(self, N, n_active):
        return self.get_shape(N, n_active)[:3]

    def tune_add(self, precision, n_min, act_min, act_max, K, L, S=0, T=0, WG=0):
        prec = _PREC_NAMES[precision] if isinstance(precision, str) else int(precision)
        self._chk(_lib.nb_tune_add(self._h, prec, int(n_min), int(act_min), int(act_max), int(K), int(L), int(S),
                                   int(T), int(WG)))

    def tune_add_batch(self, precision, kind, key_min, key_max, K, L):
        """kind 1: nbody_forces_batch keyed by mean active rows per system;
        kind 2: batched block steps keyed by mean system size."""
        prec = _PREC_NAMES[precision] if isinstance(precision, str) else int(precision)
        self._chk(_lib.nb_tune_add_batch(self._h, prec, int(kind), int(key_min), int(key_max), int(K), int(L)))

    def get_batch_launch(self, kind, key, N):
        K, L = _int(), _int()
        self._chk(_lib.nb_get_batch_launch(self._h, int(kind), int(key), int(N), ctypes.byref(K), ctypes.byref(L)))
        return K.value, L.value

    def set_split_sum(self, mode):
        """0: fixed-order two-kernel sum of the j-split (default); 1: atomic adds (the paper's alternative)."""
        self._chk(_lib.nb_set_split_sum(self._h, int(mode)))

    def tune_clear(self):
        self._chk(_lib.nb_tune_clear(self._h))

    def set_phase_timing(self, on=True):
        """Record phase events in every eager block step (``nb_set_phase_timing``)."""
        self._chk(_lib.nb_set_phase_timing(self._h, 1 if on else 0))

    def phase_times(self):
        """(schedule, forces, reduce + correct) milliseconds of the last timed
        eager block step (``nb_phase_times``); waits for that step."""
        ms = (ctypes.c_float * 3)()
        self._chk(_lib.nb_phase_times(self._h, ms))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def set_stop_source(self, stop=None):
        """Block steps read their stop tick from ``stop`` (a one-element int64
        device tensor) while it is set; None restores the argument."""
        if stop is not None:
            _check_1d(stop, 1, "stop", torch.int64, self.device)
        self._chk(_lib.nb_set_stop_source(self._h, _p(stop)))

    # ---- forces -------------------------------------------------------------
    def forces(self, pos, vel, mass, active, eps2, acc=None, jerk=None, pot=None):
        n = mass.shape[0]
        na = active.shape[0]
        _check_vec(pos, n, "pos", self.device)
        _check_vec(vel, n, "vel", self.device)
        _check_1d(mass, n, "mass", torch.float64, self.device)
        _check_1d(active, na, "active_idx", torch.int32, self.device)
        if acc is None:
            acc = torch.empty((na, 3), dtype=torch.float64, device=self.device)
        if jerk is None:
            jerk = torch.empty((na, 3), dtype=torch.float64, device=self.device)
        if pot is None:
            pot = torch.empty((na,), dtype=torch.float64, device=self.device)
        _check_vec(acc, na, "acc", self.device)
        _check_vec(jerk, na, "jerk", self.device)
        _check_1d(pot, na, "pot", torch.float64, self.device)
        self._chk(_lib.nbody_forces(self._h, _p(pos), _p(vel), _p(mass), n, _p(active), na, float(eps2),
                                    _p(acc), _p(jerk), _p(pot)))
        return acc, jerk, pot

    def forces_noalloc(self, pos, vel, mass, active, eps2, acc, jerk, pot):
        """``nbody_forces`` with the library's fixed scratch (``nbody_forces_noalloc``):
        the outputs must be given, nothing is allocated."""
        n = mass.shape[0]
        na = active.shape[0]
        _check_vec(pos, n, "pos", self.device)
        _check_vec(vel, n, "vel", self.device)
        _check_1d(mass, n, "mass", torch.float64, self.device)
        _check_1d(active, na, "active_idx", torch.int32, self.device)
        _check_vec(acc, na, "acc", self.device)
        _check_vec(jerk, na, "jerk", self.device)
        _check_1d(pot, na, "pot", torch.float64, self.device)
        self._chk(_lib.nbody_forces_noalloc(self._h, _p(pos), _p(vel), _p(mass), n, _p(active), na, float(eps2),
                                            _p(acc), _p(jerk), _p(pot)))
        return acc, jerk, pot

    def forces_ij(self, pos_j, vel_j, mass_j, pos_i, vel_i, active, eps2, acc=None, jerk=None, pot=None):
        """Forces on rows ``active`` of pos_i/vel_i from the separate j-set (``nbody_forces_ij``)."""
        nj, ni, na = mass_j.shape[0], pos_i.shape[0], active.shape[0]
        _check_vec(pos_j, nj, "pos_j", self.device)
        _check_vec(vel_j, nj, "vel_j", self.device)
        _check_1d(mass_j, nj, "mass_j", torch.float64, self.device)
        _check_vec(pos_i, ni, "pos_i", self.device)
        _check_vec(vel_i, ni, "vel_i", self.device)
        _check_1d(active, na, "active_idx", torch.int32, self.device)
        if acc is None:
            acc = torch.empty((na, 3), dtype=torch.float64, device=self.device)
        if jerk is None:
            jerk = torch.empty((na, 3), dtype=torch.float64, device=self.device)
        if pot is None:
            pot = torch.empty((na,), dtype=torch.float64, device=self.device)
        _check_vec(acc, na, "acc", self.device)
        _check_vec(jerk, na, "jerk", self.device)
        _check_1d(pot, na, "pot", torch.float64, self.device)
        self._chk(_lib.nbody_forces_ij(self._h, _p(pos_j), _p(vel_j), _p(mass_j), nj, _p(pos_i), _p(vel_i), ni,
                                       _p(active), na, float(eps2), _p(acc), _p(jerk), _p(pot)))
        return acc, jerk, pot

    # ---- sixth-order Hermite -------------------------------------------------
    def forces6(self, pos, vel, acc_j, mass, active, eps2, acc=None, jerk=None, snap=None, pot=None):
        """Acceleration, jerk, snap, potential of ``active`` (``nbody_forces6``)."""
        n, na = mass.shape[0], active.shape[0]
        _check_vec(pos, n, "pos", self.device)
        _check_vec(vel, n, "vel", self.device)
        _check_vec(acc_j, n, "acc_j", self.device)
        _check_1d(mass, n, "mass", torch.float64, self.device)
        _check_1d(active, na, "active_idx", torch.int32, self.device)
        new = lambda: torch.empty((na, 3), dtype=torch.float64, device=self.device)
        acc = new() if acc is None else acc
        jerk = new() if jerk is None else jerk
        snap = new() if snap is None else snap
        pot = torch.empty((na,), dtype=torch.float64, device=self.device) if pot is None else pot
        for t, nm in ((acc, "acc"), (jerk, "jerk"), (snap, "snap")):
            _check_vec(t, na, nm, self.device)
        _check_1d(pot, na, "pot", torch.float64, self.device)
        self._chk(_lib.nbody_forces6(self._h, _p(pos), _p(vel), _p(acc_j), _p(mass), n, _p(active), na,
                                     float(eps2), _p(acc), _p(jerk), _p(snap), _p(pot)))
        return acc, jerk, snap, pot

    def predict6(self, pos, vel, acc, jerk, snap, crackle, t_tick, t_next_tick, dt_min, pos_p, vel_p, acc_p):
        self._chk(_lib.hermite6_predict(self._h, _p(pos), _p(vel), _p(acc), _p(jerk), _p(snap), _p(crackle),
                                        _p(t_tick), int(t_next_tick), float(dt_min), pos.shape[0], _p(pos_p),
                                        _p(vel_p), _p(acc_p)))

    def correct6(self, active, acc1, jerk1, snap1, pos, vel, acc, jerk, snap, crackle, t_tick, dt_level, eta, dt_max,
                 max_level, clamp_count=None):
        self._chk(_lib.hermite6_correct(self._h, _p(active), active.shape[0], pos.shape[0], _p(acc1), _p(jerk1),
                                        _p(snap1),
                                        _p(pos), _p(vel), _p(acc), _p(jerk), _p(snap), _p(crackle), _p(t_tick),
                                        _p(dt_level), float(eta), float(dt_max), int(max_level), _p(clamp_count)))

    def startup6(self, acc, jerk, snap, eta_s, dt_max, max_level, dt_level):
        self._chk(_lib.hermite6_startup(self._h, _p(acc), _p(jerk), _p(snap), acc.shape[0], float(eta_s),
                                        float(dt_max), int(max_level), _p(dt_level)))

    def block_step6(self, N, eps2, eta, dt_max, max_level, mass, pos, vel, acc, jerk, snap, crackle, t_tick,
                    dt_level, pos_p, vel_p, acc_p, active, acc1, jerk1, snap1, pot1, sched, t_stop_tick=2 ** 63 - 1):
        self._chk(_lib.nb_block_step6(self._h, int(N), float(eps2), float(eta), float(dt_max), int(max_level),
                                      _p(mass), _p(pos), _p(vel), _p(acc), _p(jerk), _p(snap), _p(crackle),
                                      _p(t_tick), _p(dt_level), _p(pos_p), _p(vel_p), _p(acc_p), _p(active),
                                      _p(acc1), _p(jerk1), _p(snap1), _p(pot1), _p(sched), int(t_stop_tick)))

    # ---- tree code --------------------------------------------------------------
    def tree_forces(self, pos, mass, eps2, theta=0.5, n_crit=16, g_frac=1.0 / 16, acc=None, pot=None, stats=True):
        """Barnes-Hut acceleration and potential of every particle (``nb_tree_forces``).

        Returns (acc, pot, stats) with stats the numbers of cells, groups,
        accepted (group, cell) pairs, opened (group, leaf) pairs and the depth;
        with stats=False the call does not synchronise (and can be captured)
        and returns None for them."""
        n = mass.shape[0]
        _check_vec(pos, n, "pos", self.device)
        _check_1d(mass, n, "mass", torch.float64, self.device)
        acc = torch.empty((n, 3), dtype=torch.float64, device=self.device) if acc is None else acc
        pot = torch.empty((n,), dtype=torch.float64, device=self.device) if pot is None else pot
        _check_vec(acc, n, "acc", self.device)
        _check_1d(pot, n, "pot", torch.float64, self.device)
        st = (ctypes.c_int64 * 5)() if stats else None
        self._chk(_lib.nb_tree_forces(self._h, _p(pos), _p(mass), n, float(eps2), float(theta), int(n_crit),
                                      float(g_frac), _p(acc), _p(pot), st))
        if not stats:
            return acc, pot, None
        return acc, pot, dict(zip(("cells", "groups", "accepted", "opened_leaves", "depth"), list(st)))

    def tree_keys(self, pos):
        """(keys, idx): the particles' Peano-Hilbert keys in curve order and their rows (``nb_tree_keys``)."""
        n = pos.shape[0]
        _check_vec(pos, n, "pos", self.device)
        keys = torch.empty(n, dtype=torch.int64, device=self.device)
        idx = torch.empty(n, dtype=torch.int32, device=self.device)
        self._chk(_lib.nb_tree_keys(self._h, _p(pos), n, _p(keys), _p(idx)))
        return keys, idx

    def kick(self, vel, acc, h):
        """vel += h acc (``nb_kick``)."""
        n = vel.shape[0]
        _check_vec(vel, n, "vel", self.device)
        _check_vec(acc, n, "acc", self.device)
        self._chk(_lib.nb_kick(self._h, _p(vel), _p(acc), n, float(h)))

    def kick_drift(self, pos, vel, acc, h_kick, h_drift):
        """vel += h_kick acc, then pos += h_drift vel (``nb_kick_drift``)."""
        n = vel.shape[0]
        _check_vec(pos, n, "pos", self.device)
        _check_vec(vel, n, "vel", self.device)
        _check_vec(acc, n, "acc", self.device)
        self._chk(_lib.nb_kick_drift(self._h, _p(pos), _p(vel), _p(acc), n, float(h_kick), float(h_drift)))

    def forces_devcount(self, pos, vel, mass, active, n_active_dev, max_active, eps2, acc, jerk, pot):
        n = mass.shape[0]
        _check_1d(n_active_dev, 1, "n_active_dev", torch.int32, self.device)
        self._chk(_lib.nbody_forces_devcount(self._h, _p(pos), _p(vel), _p(mass), n, _p(active), _p(n_active_dev),
                                             int(max_active), float(eps2), _p(acc), _p(jerk), _p(pot)))
        return acc, jerk, pot

    def time_forces(self, K, L, S, pos, vel, mass, active, eps2, acc, jerk, pot, reps=5, T=0, WG=0):
        ms = _dbl()
        self._chk(_lib.nb_time_forces(self._h, int(K), int(L), int(S), int(T), int(WG), _p(pos), _p(vel), _p(mass),
                                      mass.shape[0], _p(active), active.shape[0], float(eps2), _p(acc), _p(jerk),
                                      _p(pot), int(reps), ctypes.byref(ms)))
        return ms.value

    def forces_batch(self, offsets, eps2, pos, vel, mass, active, act_offsets, acc, jerk, pot):
        """offsets, act_offsets: host int64 sequences of length C+1; eps2: host floats of length C."""
        import numpy as np
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        aoff = np.ascontiguousarray(act_offsets, dtype=np.int64)
        e2 = np.ascontiguousarray(eps2, dtype=np.float64)
        C = off.shape[0] - 1
        self._chk(_lib.nbody_forces_batch(self._h, off.ctypes.data_as(_vp), C, e2.ctypes.data_as(_vp), _p(pos),
                                          _p(vel), _p(mass), _p(active), aoff.ctypes.data_as(_vp), _p(acc),
                                          _p(jerk), _p(pot)))
        return acc, jerk, pot

    # ---- Hermite --------------------------------------------------------------
    def predict(self, pos, vel, acc, jerk, t_tick, t_next_tick, dt_min, pos_p, vel_p):
        n = pos.shape[0]
        self._chk(_lib.hermite_predict(self._h, _p(pos), _p(vel), _p(acc), _p(jerk), _p(t_tick), int(t_next_tick),
                                       float(dt_min), n, _p(pos_p), _p(vel_p)))

    def correct(self, active, pos_p, vel_p, acc1, jerk1, pos, vel, acc, jerk, t_tick, dt_level, eta, dt_max,
                max_level, clamp_dev=None):
        self._chk(_lib.hermite_correct(self._h, _p(active), active.shape[0], pos.shape[0], _p(pos_p), _p(vel_p),
                                       _p(acc1),
                                       _p(jerk1), _p(pos), _p(vel), _p(acc), _p(jerk), _p(t_tick), _p(dt_level),
                                       float(eta), float(dt_max), int(max_level), _p(clamp_dev)))

    def startup(self, acc, jerk, eta, dt_max, max_level, dt_level):
        self._chk(_lib.hermite_startup(self._h, _p(acc), _p(jerk), acc.shape[0], float(eta), float(dt_max),
                                       int(max_level), _p(dt_level)))

    def schedule(self, t_tick, dt_level, max_level, active, sched):
        self._chk(_lib.nb_schedule(self._h, _p(t_tick), _p(dt_level), t_tick.shape[0], int(max_level), _p(active),
                                   _p(sched)))

    def block_step(self, N, eps2, eta, dt_max, max_level, mass, pos, vel, acc, jerk, t_tick, dt_level, pos_p, vel_p,
                   active, acc1, jerk1, pot1, sched, t_stop_tick=2 ** 63 - 1):
        self._chk(_lib.nb_block_step(self._h, int(N), float(eps2), float(eta), float(dt_max), int(max_level),
                                     _p(mass), _p(pos), _p(vel), _p(acc), _p(jerk), _p(t_tick), _p(dt_level),
                                     _p(pos_p), _p(vel_p), _p(active), _p(acc1), _p(jerk1), _p(pot1), _p(sched),
                                     int(t_stop_tick)))

    def block_step_batch(self, offsets, eps2, eta, dt_max, max_level, mass, pos, vel, acc, jerk, t_tick, dt_level,
                         pos_p, vel_p, active, acc1, jerk1, pot1, sched, t_stop_tick=2 ** 63 - 1):
        """offsets (C+1) and eps2 (C): host int64/float64 arrays (kept alive by the caller)."""
        import numpy as np
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        e2 = np.ascontiguousarray(eps2, dtype=np.float64)
        self._chk(_lib.nb_block_step_batch(self._h, off.ctypes.data_as(_vp), off.shape[0] - 1,
                                           e2.ctypes.data_as(_vp), float(eta), float(dt_max), int(max_level),
                                           _p(mass), _p(pos), _p(vel), _p(acc), _p(jerk), _p(t_tick), _p(dt_level),
                                           _p(pos_p), _p(vel_p), _p(active), _p(acc1), _p(jerk1), _p(pot1),
                                           _p(sched), int(t_stop_tick)))

    def energy(self, pos, vel, mass, pot, out):
        self._chk(_lib.nb_energy(self._h, _p(pos), _p(vel), _p(mass), _p(pot), mass.shape[0], _p(out)))
        return out


# Function-style aliases with the C names (the context is the first argument).
def nbody_forces(ctx, pos, vel, mass, active_idx, eps2, acc=None, jerk=None, pot=None):
    return ctx.forces(pos, vel, mass, active_idx, eps2, acc, jerk, pot)


def nbody_forces_noalloc(ctx, pos, vel, mass, active_idx, eps2, acc, jerk, pot):
    return ctx.forces_noalloc(pos, vel, mass, active_idx, eps2, acc, jerk, pot)


def nbody_forces_devcount(ctx, *a, **k):
    return ctx.forces_devcount(*a, **k)


def nbody_forces_batch(ctx, *a, **k):
    return ctx.forces_batch(*a, **k)


def hermite_predict(ctx, *a, **k):
    return ctx.predict(*a, **k)


def hermite_correct(ctx, *a, **k):
    return ctx.correct(*a, **k)


def hermite_startup(ctx, *a, **k):
    return ctx.startup(*a, **k)


def nb_schedule(ctx, *a, **k):
    return ctx.schedule(*a, **k)


def nb_block_step(ctx, *a, **k):
    return ctx.block_step(*a, **k)


def nb_energy(ctx, *a, **k):
    return ctx.energy(*a, **k)


def version():
    return _lib.nb_version().decode()


def nbody_forces_ij(ctx, *a, **k):
    return ctx.forces_ij(*a, **k)


def nb_kick(ctx, *a, **k):
    return ctx.kick(*a, **k)


def nb_kick_drift(ctx, *a, **k):
    return ctx.kick_drift(*a, **k)


def nbody_forces6(ctx, *a, **k):
    return ctx.forces6(*a, **k)


def hermite6_predict(ctx, *a, **k):
    return ctx.predict6(*a, **k)


def hermite6_correct(ctx, *a, **k):
    return ctx.correct6(*a, **k)


def hermite6_startup(ctx, *a, **k):
    return ctx.startup6(*a, **k)


def nb_block_step6(ctx, *a, **k):
    return ctx.block_step6(*a, **k)


def nb_tree_forces(ctx, *a, **k):
    return ctx.tree_forces(*a, **k)


def nb_sync(ctx):
    return ctx.sync()
