"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in a copy of the oracle (on the CPU only) -- a dropped term, a
wrong sign, power, constant or index -- and runs the pin tests against the
copy, which must fail."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "forces.c")

# (name, regex, replacement): applied to every match, i.e. to both the
# double and the extended-precision evaluation.
FORCE_MUTANTS = [
    ("jerk factor 3 -> 2", r"3\.0L? \* ru", "2.0 * ru"),
    ("jerk sign", r"\(ux - c \* rx\)", "(ux + c * rx)"),
    ("acc power s^-1 instead of s^-3/2", r"\* inv_sqrt_s \* inv_s;", "* inv_s;"),
    ("potential sign", r"ph -= ", "ph += "),
    ("softening dropped", r" \+ \(long double\)eps2;| \+ eps2;", ";"),
    ("y/z component swap", r"pos\[3 \* j \+ 1\] - yi", "pos[3 * j + 2] - yi"),
    ("self pair not excluded", r"if \(j == i\) continue;", ""),
    ("relative velocity uses i twice", r"vel\[3 \* j\] - vxi", "vel[3 * i] - vxi"),
    ("jerk uses acc direction only", r"\(uz - c \* rz\)", "(uz - c * rx)"),
]


def _build_mutant(tmp_path, name, pat, rep):
    src = open(SRC).read()
    mut, n = re.subn(pat, rep, src)
    assert n > 0, f"mutation {name!r} did not apply"
    c = tmp_path / "forces_mut.c"
    c.write_text(mut)
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", str(c), "-o", str(so),
                    "-lm"], check=True)
    return so


@pytest.mark.slow
@pytest.mark.parametrize("name,pat,rep", FORCE_MUTANTS, ids=[m[0] for m in FORCE_MUTANTS])
def test_force_pins_catch_mutant(tmp_path, name, pat, rep):
    so = _build_mutant(tmp_path, name, pat, rep)
    env = dict(os.environ, NB_ORACLE_LIB=str(so), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_forces.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 1, f"mutant {name!r} survived:\n{r.stdout[-2000:]}"


# Mutants that the 50-digit brute-force pin alone must catch (it runs by itself
# against each of them).
BRUTE_FORCE_MUTANTS = [
    ("i's mass weights the acceleration", r"mass\[j\] \* inv_sqrt_s \* inv_s;", "mass[i] * inv_sqrt_s * inv_s;"),
    ("r.u takes u_y for u_z", r"rz \* uz;", "rz * uy;"),
    ("last j dropped", r"int64_t j = 0; j < n;", "int64_t j = 0; j < n - 1;"),
    ("softening counted twice", r" \+ \(long double\)eps2;| \+ eps2;", " + 2 * eps2;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,pat,rep", BRUTE_FORCE_MUTANTS, ids=[m[0] for m in BRUTE_FORCE_MUTANTS])
def test_brute_force_pin_catches_mutant(tmp_path, name, pat, rep):
    so = _build_mutant(tmp_path, name, pat, rep)
    env = dict(os.environ, NB_ORACLE_LIB=str(so), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_forces.py") + "::test_mpmath_brute_force_small_sets"],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 1, f"mutant {name!r} survived the brute-force pin:\n{r.stdout[-2000:]}"


# Hermite mutants: patch one function of oracle.hermite and run a pin.
def _hermite_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_oracle_hermite as T
    return [T.test_predictor_exact_for_constant_jerk, T.test_corrector_exact_for_cubic_acceleration,
            T.test_aarseth_hand_value, T.test_level_rules, T.test_block_step_invariants]


def _mut_predict(x, v, a, j, d):
    d = np.asarray(d, dtype=np.float64)
    d = d[:, None] if d.ndim == 1 else d
    return x + v * d + a * (d * d / 2.0) + j * (d * d * d / 2.0), v + a * d + j * (d * d / 2.0)


def _mut_interpolate(a0, j0, a1, j1, dt):
    dt = np.asarray(dt, dtype=np.float64)
    dt = dt[:, None] if dt.ndim == 1 else dt
    a2 = (-6.0 * (a0 - a1) - dt * (4.0 * j1 + 2.0 * j0)) / (dt * dt)   # j0/j1 transposed
    a3 = (12.0 * (a0 - a1) + 6.0 * dt * (j0 + j1)) / (dt * dt * dt)
    return a2, a3


def _mut_correct(xp, vp, a2, a3, dt):
    dt = np.asarray(dt, dtype=np.float64)
    dt = dt[:, None] if dt.ndim == 1 else dt
    return xp + a2 * dt ** 4 / 24.0 + a3 * dt ** 5 / 24.0, vp + a2 * dt ** 3 / 6.0 + a3 * dt ** 4 / 24.0


def _mut_aarseth(a1, j1, a2, a3, dt, eta, dt_max):
    from oracle import hermite as H
    n = lambda u: np.sqrt((u * u).sum(-1))
    num = n(a1) * n(a2) + n(j1) ** 2            # a2 at the start instead of the end of the step
    den = n(j1) * n(a3) + n(a2) ** 2
    return np.where(den > 0, np.sqrt(eta * num / np.where(den > 0, den, 1)), dt_max)


def _mut_new_level(level, dt_star, t_new, dt_max, max_level):
    level = np.array(level, dtype=np.int64)
    out = level.copy()
    for k in range(level.size):
        L = int(level.flat[k]); ds = float(np.asarray(dt_star).flat[k]); dt = dt_max * 2.0 ** -L
        if ds < dt:
            while dt > ds and L < max_level:
                L += 1; dt = dt_max * 2.0 ** -L
        elif ds >= 2.0 * dt and L > 0:
            L -= 1                               # doubles without the commensurability check
        out.flat[k] = L
    return out, np.zeros(level.shape, dtype=bool)


HERMITE_MUTANTS = [("predictor jerk coefficient", "predict", _mut_predict),
                   ("interpolation j0/j1 transposed", "interpolate", _mut_interpolate),
                   ("corrector a3 coefficient", "correct", _mut_correct),
                   ("Aarseth uses start-of-step a2", "aarseth_dt", _mut_aarseth),
                   ("level doubling not commensurate", "new_level", _mut_new_level)]


@pytest.mark.slow
@pytest.mark.parametrize("name,attr,fn", HERMITE_MUTANTS, ids=[m[0] for m in HERMITE_MUTANTS])
def test_hermite_pins_catch_mutant(monkeypatch, name, attr, fn):
    from oracle import hermite as H
    monkeypatch.setattr(H, attr, fn)
    caught = False
    for pin in _hermite_pins():
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived every Hermite pin"


def _mut_energy_L_reversed(pos, vel, mass, pot):
    e = _ENERGY(pos, vel, mass, pot)
    e["L"] = (mass[:, None] * np.cross(vel, pos)).sum(0)     # v x x instead of x x v
    return e


def _mut_energy_no_half_W(pos, vel, mass, pot):
    e = _ENERGY(pos, vel, mass, pot)
    e["W"] = 2.0 * e["W"]                                    # every pair counted twice
    e["E"] = e["K"] + e["W"]
    return e


def _mut_energy_P_unweighted(pos, vel, mass, pot):
    e = _ENERGY(pos, vel, mass, pot)
    e["P"] = vel.sum(0)
    return e


def _mut_energy_L_unweighted(pos, vel, mass, pot):
    e = _ENERGY(pos, vel, mass, pot)
    e["L"] = np.cross(pos, vel).sum(0)
    return e


from oracle.hermite import energy as _ENERGY  # noqa: E402

ENERGY_MUTANTS = [("angular momentum v x x", _mut_energy_L_reversed),
                  ("potential energy without the half", _mut_energy_no_half_W),
                  ("momentum without masses", _mut_energy_P_unweighted),
                  ("angular momentum without masses", _mut_energy_L_unweighted)]


@pytest.mark.parametrize("name,fn", ENERGY_MUTANTS, ids=[m[0] for m in ENERGY_MUTANTS])
def test_energy_pins_catch_mutant(monkeypatch, name, fn):
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_oracle_hermite as T
    from oracle import hermite as H
    monkeypatch.setattr(H, "energy", fn)
    caught = False
    for pin in (T.test_energy_circular_two_body_closed_form, T.test_energy_rotated_and_boosted_pair):
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived the energy pins"


# Bridge mutants: patch one function of oracle.bridge and run its pins.
def _bridge_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_oracle_bridge as T
    return [T.test_cross_field_adds_up_to_the_whole, T.test_kicks_conserve_total_momentum_and_keep_positions,
            T.test_two_body_split_is_the_textbook_leapfrog, T.test_two_body_split_converges_at_second_order,
            T.test_massless_cluster_leaves_the_galaxy_a_plain_leapfrog,
            T.test_cluster_in_galaxy_converges_at_second_order_in_the_bridge_step,
            T.test_tree_cross_field_at_theta_zero_is_the_direct_bridge,
            T.test_tree_cross_field_conserves_energy_and_needs_one_softening]


def _mut_step_first_order(st):
    from oracle import bridge as B
    B.kick(st, st.dt)                      # the whole kick before the drifts
    B.drift_cluster(st)
    if st.mg.shape[0]:
        B.drift_galaxy(st)
    st.steps += 1
    return st


def _mut_cross_sign(x_i, v_i, x_j, v_j, m_j, eps2):
    from oracle import forces_f64
    nj, ni = np.asarray(m_j).shape[0], np.asarray(x_i).shape[0]
    a, j, p, _ = forces_f64(np.concatenate([x_j, x_i]), np.concatenate([v_j, v_i]),
                            np.concatenate([m_j, np.zeros(ni)]), eps2, np.arange(nj, nj + ni, dtype=np.int32))
    return -a, -j, p


def _mut_kick_c_only(st, h):
    from oracle import bridge as B
    c = st.cluster
    c.v = c.v + h * B.cross_forces(c.x, c.v, st.xg, st.vg, st.mg, st.eps2_gc)[0]


def _mut_galaxy_drift_first(st):
    from oracle import bridge as B
    h = st.dt / st.n_sub
    for _ in range(st.n_sub):
        st.xg = st.xg + h * st.vg          # drift before the half kick
        st.vg = st.vg + (0.5 * h) * st.ag
        st.ag = st.field(st.xg, st.mg)
        st.vg = st.vg + (0.5 * h) * st.ag


def _mut_cross_includes_receivers(x_i, v_i, x_j, v_j, m_j, eps2):
    from oracle import forces_f64
    nj, ni = np.asarray(m_j).shape[0], np.asarray(x_i).shape[0]
    # receivers keep a mass: they pull on each other too
    mass = np.concatenate([m_j, np.full(ni, float(np.mean(m_j)) if nj else 0.0)])
    a, j, p, _ = forces_f64(np.concatenate([x_j, x_i]), np.concatenate([v_j, v_i]), mass, eps2,
                            np.arange(nj, nj + ni, dtype=np.int32))
    return a, j, p


def _mut_tree_cross_c_massive(xg, mg, xc, eps2, theta, n_crit=16, g_frac=1.0 / 16):
    from oracle import tree as TR
    ng = np.asarray(mg).shape[0]
    x = np.concatenate([xg, xc])
    # c keeps a mass in the tree: it pulls on g and on itself
    m = np.concatenate([mg, np.full(np.asarray(xc).shape[0], float(np.mean(mg)))])
    t = TR.build(x, m, n_crit)
    a = TR.forces(x, m, eps2, theta, n_crit, g_max=g_frac * t.side, tree=t)[0]
    return a[:ng], a[ng:]


BRIDGE_MUTANTS = [("whole kick first (first-order split)", "step", _mut_step_first_order),
                  ("cross field sign", "cross_forces", _mut_cross_sign),
                  ("g never kicked", "kick", _mut_kick_c_only),
                  ("galaxy drifts before its half kick", "drift_galaxy", _mut_galaxy_drift_first),
                  ("receivers exert forces", "cross_forces", _mut_cross_includes_receivers),
                  ("c exerts in the tree cross field", "galaxy_and_cross_tree", _mut_tree_cross_c_massive)]


@pytest.mark.slow
@pytest.mark.parametrize("name,attr,fn", BRIDGE_MUTANTS, ids=[m[0] for m in BRIDGE_MUTANTS])
def test_bridge_pins_catch_mutant(monkeypatch, name, attr, fn):
    from oracle import bridge as B
    monkeypatch.setattr(B, attr, fn)
    caught = False
    for pin in _bridge_pins():
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived every bridge pin"


# Snap mutants: planted in a copy of oracle/snap.c, run against its pins.
SNAP_SRC = os.path.join(ROOT, "oracle", "snap.c")
SNAP_MUTANTS = [
    ("snap u-term factor 6 -> 3", r"6\.0L \* ru \* u\[c\]", "3.0L * ru * u[c]"),
    ("snap last-term factor 15 -> 5", r"15\.0L \* ru \* ru", "5.0L * ru * ru"),
    ("snap r.w term dropped", r"\(uu \+ rw\)", "(uu)"),
    ("snap relative acceleration sign", r"\(long double\)accj\[3 \* j \+ c\] - \(long double\)accj\[3 \* i \+ c\]",
     "(long double)accj[3 * i + c] - (long double)accj[3 * j + c]"),
    ("snap power s^-5/2 -> s^-3/2 in the r-term", r"\(uu \+ rw\) \* r\[c\] / s52", "(uu + rw) * r[c] / s32"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,pat,rep", SNAP_MUTANTS, ids=[m[0] for m in SNAP_MUTANTS])
def test_snap_pins_catch_mutant(tmp_path, name, pat, rep):
    src = open(SNAP_SRC).read()
    mut, n = re.subn(pat, rep, src)
    assert n > 0, f"mutation {name!r} did not apply"
    c = tmp_path / "snap_mut.c"
    c.write_text(mut)
    so = tmp_path / "liboracle_snap_mut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", str(c), "-o", str(so),
                    "-lm"], check=True)
    env = dict(os.environ, NB_ORACLE_SNAP_LIB=str(so), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_hermite6.py")],
                       env=env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 1, f"mutant {name!r} survived:\n{r.stdout[-2000:]}"


# 6th-order Hermite mutants: patch one function of oracle.hermite6.
def _hermite6_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_oracle_hermite6 as T
    return [T.test_interpolation_recovers_a_quintic, T.test_corrector_exact_for_quintic_acceleration,
            T.test_predictor_exact_for_constant_crackle, T.test_step_criterion_hand_values,
            T.test_kepler_sixth_order_convergence, T.test_block_step_invariants_and_energy]


def _m6_predict(x, v, a, j, s, c, d):
    d = np.asarray(d, dtype=np.float64)
    d = d[:, None] if d.ndim == 1 else d
    return (x + v * d + a * d ** 2 / 2 + j * d ** 3 / 6 + s * d ** 4 / 24 + c * d ** 5 / 24,   # crackle /24
            v + a * d + j * d ** 2 / 2 + s * d ** 3 / 6 + c * d ** 4 / 24,
            a + j * d + s * d ** 2 / 2 + c * d ** 3 / 6)


def _m6_interpolate(a0, j0, s0, a1, j1, s1, dt):
    from oracle import hermite6 as H6
    return H6.__dict__["_orig_interpolate"](a0, s0, j0, a1, j1, s1, dt)       # j0/s0 swapped


def _m6_correct(x0, v0, a0, j0, s0, c0, p0, q0, dt):
    dt = np.asarray(dt, dtype=np.float64)
    dt = dt[:, None] if dt.ndim == 1 else dt
    v1 = v0 + a0 * dt + j0 * dt ** 2 / 2 + s0 * dt ** 3 / 6 + c0 * dt ** 4 / 24 + p0 * dt ** 5 / 120
    x1 = x0 + v0 * dt + a0 * dt ** 2 / 2 + j0 * dt ** 3 / 6 + s0 * dt ** 4 / 24 + c0 * dt ** 5 / 120 \
        + p0 * dt ** 6 / 720                                                   # q0 terms dropped
    return x1, v1, c0 + p0 * dt + q0 * dt ** 2 / 2, p0 + q0 * dt


def _m6_new_dt(a1, j1, s1, c1, p1, q, eta, dt_max):
    n = lambda u: np.sqrt((u * u).sum(-1))
    num = np.sqrt(n(a1) * n(s1)) + n(j1)
    den = np.sqrt(n(c1) * n(q)) + n(p1)
    return np.where(den > 0, eta * np.sqrt(num / np.where(den > 0, den, 1)), dt_max)   # exponent 1/2


def _m6_startup(a, j, s, eta_s, dt_max, max_level):
    from oracle import hermite as H
    return H.startup_level(a, j, eta_s, dt_max, max_level)                     # snap term ignored


HERMITE6_MUTANTS = [("predictor crackle coefficient", "predict", _m6_predict),
                    ("interpolation j0/s0 swapped", "interpolate", _m6_interpolate),
                    ("corrector drops the fifth derivative", "correct", _m6_correct),
                    ("step criterion exponent 1/2", "new_dt", _m6_new_dt),
                    ("start-up ignores the snap", "startup_level", _m6_startup)]


@pytest.mark.slow
@pytest.mark.parametrize("name,attr,fn", HERMITE6_MUTANTS, ids=[m[0] for m in HERMITE6_MUTANTS])
def test_hermite6_pins_catch_mutant(monkeypatch, name, attr, fn):
    from oracle import hermite6 as H6
    monkeypatch.setitem(H6.__dict__, "_orig_interpolate", H6.interpolate)
    monkeypatch.setattr(H6, attr, fn)
    caught = False
    for pin in _hermite6_pins():
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived every 6th-order pin"


# Tree-code mutants: patch one function of oracle.tree and run its pins.
def _tree_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_oracle_tree as T
    return [lambda: T.test_hilbert_keys_are_a_bijection_along_unit_steps(3), T.test_hilbert_prefixes_are_aligned_cubes,
            T.test_tree_leaves_partition_and_cubes_contain, T.test_moments_definitions_and_parallel_axis,
            T.test_multipole_far_field_error_falls_as_the_fifth_power,
            T.test_opening_criterion_never_accepts_a_cell_touching_its_group, T.test_groups_are_contiguous_and_small,
            T.test_theta_zero_is_the_direct_sum]


def _mt_keys_no_gray(ijk, bits=21):
    from oracle import tree as TR
    # the keys of the axes themselves (a Morton order): loses the unit steps
    key = np.zeros(ijk.shape[0], dtype=np.int64)
    for b in range(bits - 1, -1, -1):
        for k in range(3):
            key = (key << 1) | ((ijk[:, k].astype(np.int64) >> b) & 1)
    return key


def _mt_accept(cell, glo, ghi, theta):
    gap = np.maximum(np.maximum(cell.corner - ghi, glo - (cell.corner + cell.side)), 0.0)
    return theta * float(gap @ gap) > cell.side * cell.side                # theta not squared


def _mt_field(M, X, Q, x, eps2):
    y = x - X
    s = (y * y).sum(1) + eps2
    Qy = y @ Q.T
    yQy = (y * Qy).sum(1)
    a = -M * y * s[:, None] ** -1.5 - Qy * s[:, None] ** -2.5 + 2.5 * (yQy * s ** -3.5)[:, None] * y   # sign
    return a, -M * s ** -0.5 - 0.5 * yQy * s ** -2.5


def _mt_moments(x, m, centre):
    M = float(m.sum())
    X = (m[:, None] * x).sum(0) / M if M > 0 else centre
    d = x - X
    dd = (d * d).sum(1)
    Q = (m[:, None, None] * (2.0 * (d[:, :, None] * d[:, None, :]) - dd[:, None, None] * np.eye(3))).sum(0)
    return M, X, Q                                                          # factor 3 -> 2


def _mt_groups(tree, g_max, size=64):
    n = tree.mass.shape[0]
    return [(b, min(n, b + size)) for b in range(0, n, size)]            # never split


TREE_MUTANTS = [("Morton keys instead of Hilbert", "hilbert_keys", _mt_keys_no_gray),
                ("opening criterion without theta squared", "_accept", _mt_accept),
                ("quadrupole force sign", "cell_field", _mt_field),
                ("quadrupole factor 3 -> 2", "moments", _mt_moments),
                ("groups never split", "groups", _mt_groups)]


@pytest.mark.slow
@pytest.mark.parametrize("name,attr,fn", TREE_MUTANTS, ids=[m[0] for m in TREE_MUTANTS])
def test_tree_pins_catch_mutant(monkeypatch, name, attr, fn):
    from oracle import tree as TR
    monkeypatch.setattr(TR, attr, fn)
    caught = False
    for pin in _tree_pins():
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived every tree pin"


# Generator mutants: one mistake planted in a copy of the synth source, loaded
# as its own module whose functions replace synth's for the pins.
SYNTH_SRC = os.path.join(ROOT, "synth", "__init__.py")
SYNTH_MUTANTS = [
    ("Plummer radius exponent -1/2", r"np\.power\(x, -2\.0 / 3\.0\)", "np.power(x, -0.5)"),
    ("Plummer speed density exponent 5/2", r"np\.power\(1\.0 - qq \* qq, 3\.5\)", "np.power(1.0 - qq * qq, 2.5)"),
    ("Plummer escape factor sqrt(2) dropped", r"speed = q \* np\.sqrt\(2\.0\) \*", "speed = q *"),
    ("Plummer length unit not scaled", r"pos \*= 3\.0 \* np\.pi / 16\.0", "pos *= 1.0"),
    ("Hernquist radius X/(1-X)", r"r = sx / \(1\.0 - sx\)", "r = x / (1.0 - x)"),
    ("Hernquist dispersion without 1/sqrt(3)", r"sig = np\.sqrt\(r\) / \(1\.0 \+ r\) / np\.sqrt\(3\.0\)",
     "sig = np.sqrt(r) / (1.0 + r)"),
    ("i-set selection on squared distance", r"sel \|= np\.sqrt\(\(d \* d\)\.sum\(1\)\) < r_sel", "sel |= (d * d).sum(1) < r_sel"),
    ("cluster sizes uniform instead of log-uniform",
     r"np\.floor\(n_min \* np\.power\(n_max / n_min, u\)\)", "np.floor(n_min + (n_max - n_min) * u)"),
]


def _synth_pins():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import test_synth as T
    return [lambda: T.test_plummer_radii_follow_the_truncated_cumulative_mass(3),
            lambda: T.test_plummer_energies_and_virial_ratio(3),
            T.test_hernquist_galaxies_cumulative_mass_and_dispersion,
            T.test_merger_i_set_size_and_membership,
            T.test_cluster_batch_sizes_softening_and_clusters]


@pytest.mark.slow
@pytest.mark.parametrize("name,pat,rep", SYNTH_MUTANTS, ids=[m[0] for m in SYNTH_MUTANTS])
def test_synth_pins_catch_mutant(monkeypatch, name, pat, rep):
    import types
    import synth
    src, n = re.subn(pat, rep, open(SYNTH_SRC).read())
    assert n > 0, f"mutation {name!r} did not apply"
    mod = types.ModuleType("synth_mutant")
    exec(compile(src, "synth_mutant", "exec"), mod.__dict__)
    for attr in ("plummer", "cluster_batch", "hernquist_merger"):
        monkeypatch.setattr(synth, attr, getattr(mod, attr))
    caught = False
    for pin in _synth_pins():
        try:
            pin()
        except AssertionError:
            caught = True
            break
    assert caught, f"mutant {name!r} survived every generator pin"
