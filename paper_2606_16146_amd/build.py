"""Compiles the HIP library libzc.so for gfx950 (in-tree, next to this file).

The round kernels of each gate are instantiated in their own translation unit
(zc_inst.hip built once per gate), and all units compile in parallel.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libzc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]

# (source, extra defines, object name)
UNITS = [("zc_api.hip", [], "zc_api.o"), ("zc_testing.hip", [], "zc_testing.o"),
         ("zc_inst.hip", ["-DZC_INST_VANILLA"], "zc_inst_vanilla.o")]
UNITS += [("zc_inst.hip", [f"-DZC_INST_PROD={m}"], f"zc_inst_prod{m}.o") for m in range(1, 9)]
# the polynomials of Table 1, m = P + 16 A
UNITS += [("zc_inst.hip", [f"-DZC_INST_SUM={c}"], f"zc_inst_sum{c}.o") for c in (2, 18, 34, 50, 3, 4)]


def _compile(unit, verbose):
    src, defs, obj = unit
    cmd = [HIPCC, *FLAGS, *defs, "-c", "-o", os.path.join(BUILD, obj), os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src} {defs}:\n" + res.stderr[-8000:])
    return os.path.join(BUILD, obj)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4, len(UNITS))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr[-8000:])
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
