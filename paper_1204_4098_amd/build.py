"""Build the HIP library liblbm_hip.so in-tree for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm_hip.so")
# index-checked build of the same sources (every global access checked against
# its buffer; see LBM_CHECK_INDEX in csrc/lbm_kernels.hpp), for the tests
LIB_CHECK = os.path.join(HERE, "liblbm_hip_check.so")
SOURCES = ["lbm_lib.hip", "thermo.cpp", "mlp.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast-honor-pragmas", "-munsafe-fp-atomics"]


def _compile(src: str, obj: str, extra, verbose: bool) -> subprocess.Popen:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    path = os.path.join(CSRC, src)
    if src.endswith(".cpp"):
        cmd = [hipcc, "-x", "c++", "-O2", "-std=c++17", "-fPIC", "-Wall",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", path, "-o", obj]
    else:
        cmd = [hipcc, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd)


def _link(lib: str, objs, verbose: bool) -> None:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp", *objs]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False, check: bool = True) -> str:
    """Compile the library in-tree; with check=True also the index-checked
    variant (only lbm_lib.hip differs: it is compiled a second time with
    LBM_CHECK_INDEX; the other objects are shared).  Returns the release path."""
    objs = {src: os.path.join(CSRC, src + ".o") for src in SOURCES}
    jobs = [(_compile(src, obj, [], verbose), obj) for src, obj in objs.items()]
    chk_obj = os.path.join(CSRC, "lbm_lib.hip.check.o")
    if check:
        jobs.append((_compile("lbm_lib.hip", chk_obj, ["-DLBM_CHECK_INDEX"], verbose), chk_obj))
    failed = [obj for p, obj in jobs if p.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    _link(LIB, list(objs.values()), verbose)
    if check:
        _link(LIB_CHECK, [chk_obj] + [o for s, o in objs.items() if s != "lbm_lib.hip"], verbose)
    for _, obj in jobs:
        os.remove(obj)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, check="--release-only" not in sys.argv))
