"""Build libxod.so (HIP for gfx950) in-tree with hipcc.

    python paper_2512_06729_amd/build.py   (a plain script: importing the
    package itself needs the built library)

Every call recompiles.  Packed-FP32 instruction selection is disabled for
all device code.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libxod.so")
ARCH = os.environ.get("XOD_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "k_chem.hip", "k_btd.hip", "k_mixed.hip", "k_step.hip", "k_cr.hip", "k_photo.hip",
           "cr.cpp", "batch.cpp", "prof.cpp", "serve.cpp", "parcel.cpp", "tune.cpp"]

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[-1] if cmd else ''}")
    return r


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc] + HIP_FLAGS + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, obj))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "4"))))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocblas"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
