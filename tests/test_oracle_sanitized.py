"""The C oracle under the host sanitizers: oracle/forces.c and oracle/snap.c
built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, CPU only),
and the force and snap pins run against those builds.  Any out-of-bounds
access, use of freed memory or undefined operation in the oracle's C code
aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-std=c11"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_force_and_snap_pins_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    libs = {}
    for src, env_key in (("forces.c", "NB_ORACLE_LIB"), ("snap.c", "NB_ORACLE_SNAP_LIB")):
        out = tmp_path / (src[:-2] + "_san.so")
        subprocess.run(["gcc", *FLAGS, os.path.join(ROOT, "oracle", src), "-o", str(out), "-lm"], check=True)
        libs[env_key] = str(out)
    env = dict(os.environ, PYTHONPATH=ROOT, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               # the Python interpreter itself is not built for leak checking
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1", **libs)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_forces.py"),
                        os.path.join(ROOT, "tests", "test_oracle_hermite6.py"), "-k", "not slow"],
                       env=env, capture_output=True, text=True, cwd=ROOT, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


@pytest.mark.slow
def test_sanitized_build_catches_a_planted_overrun(tmp_path):
    # The same harness on a copy of forces.c whose j loop runs one past the
    # end: AddressSanitizer must stop the run.
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    src = open(os.path.join(ROOT, "oracle", "forces.c")).read()
    bad = src.replace("for (int64_t j = 0; j < n; ++j) {", "for (int64_t j = 0; j <= n; ++j) {", 1)
    assert bad != src
    c = tmp_path / "forces_overrun.c"
    c.write_text(bad)
    so = tmp_path / "forces_overrun.so"
    subprocess.run(["gcc", *FLAGS, str(c), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, PYTHONPATH=ROOT, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", NB_ORACLE_LIB=str(so))
    code = ("import numpy as np, oracle; p = np.random.default_rng(1).random((50, 3)); "
            "oracle.forces_f64(p, p, np.ones(50), 1e-3)")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, (r.returncode, r.stderr[-2000:])
