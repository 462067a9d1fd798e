"""Error measures used by the parity tests (numpy, float64).

Per particle i with reference value a_i and magnitude sum A_i = sum_j |a_ij|:
  rel_i  = |da_i| / |a_i|           (the relative error the gates name)
  cond_i = |da_i| / A_i             (error on the scale that rounding sets)
and over all rows: the RMS and max of rel_i, and the normwise
||da|| / ||a||.
"""
import numpy as np


def vec_err(got, ref, absum):
    got = np.asarray(got, dtype=np.float64).reshape(ref.shape)
    d = got - ref
    if ref.ndim == 2:
        dn = np.linalg.norm(d, axis=1)
        rn = np.linalg.norm(ref, axis=1)
    else:
        dn = np.abs(d)
        rn = np.abs(ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(rn > 0, dn / rn, np.where(dn > 0, np.inf, 0.0))
        cond = np.where(absum > 0, dn / absum, np.where(dn > 0, np.inf, 0.0))
    normwise = float(np.linalg.norm(d) / np.linalg.norm(ref)) if np.linalg.norm(ref) > 0 else float(np.linalg.norm(d))
    return dict(rms=float(np.sqrt(np.mean(rel ** 2))) if rel.size else 0.0,
                max=float(rel.max()) if rel.size else 0.0,
                median=float(np.median(rel)) if rel.size else 0.0,
                cond_max=float(cond.max()) if cond.size else 0.0,
                normwise=normwise)


def all_errs(acc, jerk, pot, ref):
    return dict(acc=vec_err(acc, ref["acc"], ref["abs_acc"]),
                jerk=vec_err(jerk, ref["jerk"], ref["abs_jerk"]),
                pot=vec_err(pot, ref["pot"], ref["abs_pot"]))


# The parity gates.  FP64: per particle |da_i| <= rel |a_i| + cond A_i (A_i
# from the extended-precision oracle) and normwise <= 1e-12.  Mixed: RMS of
# the per-particle relative errors.
def check_fp64(res, ref, normwise=1e-12, rel=1e-12, cond=64 * 2.0 ** -53, names=("acc", "jerk", "pot")):
    for name, got in zip(names, res):
        r = ref[name]
        a = ref["abs_" + name]
        d = np.asarray(got) - r
        dn = np.linalg.norm(d, axis=1) if d.ndim == 2 else np.abs(d)
        rn = np.linalg.norm(r, axis=1) if r.ndim == 2 else np.abs(r)
        bound = rel * rn + cond * a
        worst = int(np.argmax(dn - bound))
        assert np.all(dn <= bound), (name, worst, dn[worst], bound[worst])
        assert np.linalg.norm(d) <= normwise * np.linalg.norm(r), name


def check_mixed(res, ref, acc_rms=1e-6, jerk_rms=1e-5, pot_rms=1e-6):
    e = all_errs(*res, ref)
    assert e["acc"]["rms"] <= acc_rms, e
    assert e["jerk"]["rms"] <= jerk_rms, e
    assert e["pot"]["rms"] <= pot_rms, e
    return e
