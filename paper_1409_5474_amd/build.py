"""Build the HIP library ``libnbody.so`` for gfx950 (in-tree).

Every HIP source is compiled with the packed-FP32 instructions switched off
(the force kernels rely on plain scalar FP32/FP64 VALU instructions) and
linked into one shared object next to this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.environ.get("NB_LIB_OUT") or os.path.join(HERE, "libnbody.so")
OBJ = os.path.join(os.path.dirname(OUT), "_build")
SOURCES = ["forces.hip", "forces6.hip", "hermite.hip", "hermite6.hip", "bridge.hip", "tree.hip", "api.hip"]
ARCH = os.environ.get("NB_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
EXTRA = os.environ.get("NB_HIPCC_EXTRA", "").split()
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", *EXTRA,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def _compile(src):
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
    noise = [ln for ln in (r.stderr or "").splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n" + "\n".join(noise))
    return obj, noise


def build(verbose: bool = False, jobs: int = 6) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for obj, noise in results:
            for ln in noise:
                print(ln)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *[o for o, _ in results], "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
