"""CPU-side checks of the C ABI: the library loads, exports every entry
point that include/nbody.h declares, and rejects bad arguments on the host
(no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char \*|void)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for need in ("nbody_forces", "hermite_predict", "hermite_correct", "nb_create", "nb_destroy",
                 "nbody_forces_batch", "nb_block_step", "nb_schedule", "nb_energy", "hermite_startup",
                 "nbody_forces_devcount", "nb_time_forces", "nb_tune_add", "nbody_forces_ij", "nb_kick",
                 "nb_kick_drift"):
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_1409_5474_amd as nb
    lib = nb.library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_string():
    import paper_1409_5474_amd as nb
    assert "gfx950" in nb.version()


def test_host_side_argument_errors_without_a_gpu():
    import paper_1409_5474_amd as nb
    lib = nb.library()
    # a NULL context is rejected before anything else
    assert lib.nbody_forces(None, None, None, None, 10, None, 1, 0.1, None, None, None) == -1
    assert lib.hermite_predict(None, None, None, None, None, None, 0, 1.0, 1, None, None) == -1
    assert lib.nb_destroy(None) == 0
    h = ctypes.c_void_p()
    # bad precision is an argument error; no device at all is a device error
    assert lib.nb_create(ctypes.byref(h), 0, 7) == -1
    rc = lib.nb_create(ctypes.byref(h), 0, 0)
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        assert rc == 0
        lib.nb_destroy(h)
    else:
        assert rc in (-3, -1)


def test_import_fails_loudly_without_the_library(tmp_path, monkeypatch):
    # The package has no CPU fallback: a missing shared object is an ImportError.
    import importlib.util
    import shutil
    pkg = tmp_path / "paper_1409_5474_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1409_5474_amd", "__init__.py"), pkg / "__init__.py")
    spec = importlib.util.spec_from_file_location("nb_copy", pkg / "__init__.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_active_range_rule_on_the_host():
    # The range test every kernel applies to an i-set entry (the library's
    # row_in_range, run here through its host entry point): [lo, hi), the
    # first bad entry reported, negative and past-the-end values caught.
    import numpy as np
    import paper_1409_5474_amd as nb
    assert nb.check_active_host(np.arange(10, dtype=np.int32), 0, 10) == -1
    assert nb.check_active_host(np.array([3, 9, 10, 2], np.int32), 0, 10) == 2
    assert nb.check_active_host(np.array([0, -1], np.int32), 0, 10) == 1
    assert nb.check_active_host(np.array([5, 4, 7], np.int32), 5, 8) == 1     # a batch system's rows [5, 8)
    assert nb.check_active_host(np.array([2 ** 31 - 1], np.int32), 0, 2 ** 31 - 1) == 0
    assert nb.check_active_host(np.zeros(0, np.int32), 0, 1) == -1
    lib = nb.library()
    assert lib.nb_check_active_host(None, 3, 0, 10, None) == -1               # null array with entries
    assert lib.nb_check_active_host(None, 0, 0, 10, None) == 0
    assert lib.nb_sync(None) == -1
