"""Build of the HIP library (libcfust.so) for gfx950 with hipcc.

The library is several translation units compiled in parallel and linked
into one shared object.  The pair kernels (fully unrolled per q and integrand
type) take most of the compile time, so their source is compiled once per
(type, range of q) group.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJ_DIR = os.path.join(HERE, "_objs")
LIB_PATH = os.path.join(HERE, "libcfust.so")

# -packed-fp32-ops: no v_pk_*_f32 from the compiler.
# -disable-machine-licm: keeps the FP64 polynomial constants of erfc and the
#   normal quantile next to their uses inside the point loop; hoisting them
#   out of the loop costs hundreds of registers and spills.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-disable-machine-licm",
]

# (object name, source, extra defines)
PAIR_GROUPS = [(1, 3), (4, 4), (5, 5), (6, 6), (7, 8), (9, 10), (11, 12)]
UNITS = [
    ("cfust_capi", "cfust_capi.hip", []),
    ("cfust_batched", "cfust_batched.hip", []),
    ("cfust_surrogate", "cfust_surrogate.hip", []),
] + [
    (f"cfust_pairs_{tn}_q{lo}_{hi}", "cfust_pairs.hip",
     [f"-DCFUST_PAIRS_T={t}", f"-DCFUST_PAIRS_QLO={lo}", f"-DCFUST_PAIRS_QHI={hi}"])
    for t, tn in (("double", "f64"), ("float", "f32")) for lo, hi in PAIR_GROUPS
]


def _sources_mtime() -> float:
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC)
             if f.endswith((".hip", ".hpp"))] + [os.path.join(INCLUDE, "cfust.h"), __file__]
    return max(os.path.getmtime(p) for p in paths)


def _compile(hipcc: str, unit, verbose: bool, force: bool, newest: float) -> str:
    name, src, defs = unit
    obj = os.path.join(OBJ_DIR, name + ".o")
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
        return obj
    cmd = [hipcc] + HIPCC_FLAGS + defs + ["-c", "-o", obj + ".tmp", os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed for {name}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(verbose: bool = False, force: bool = True, jobs: int | None = None) -> str:
    """Compile every unit (all of them when force, else those older than a
    source) and link libcfust.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    newest = _sources_mtime()
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(jobs) as pool:
        objs = list(pool.map(lambda u: _compile(hipcc, u, verbose, force, newest), UNITS))
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link failed for libcfust.so")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True, force="--incremental" not in sys.argv))
