"""Build the HIP library libvplbm.so and the measurement probes libvplbm_probes.so for gfx950
(MI355X) in-tree.

    python -m paper_1812_05401_amd.build [-v]

hipcc cross-compiles without a GPU.  Packed-FP32 instructions are disabled on the device pass.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libvplbm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "runtime.hip", "pool.hip", "static_scratch.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "lattice.hpp", "internal.hpp", "pool_policy.hpp", "step_plan.hpp", "static_scratch.hpp")] + [
    os.path.join(INCLUDE, "vplbm.h")]
ARCH = os.environ.get("VPLBM_OFFLOAD_ARCH", "gfx950")
# The probes: the step's access patterns with a trivial update, a copy, FMA chains (bench.py).
PROBE_LIB = os.path.join(PKG, "libvplbm_probes.so")
PROBE_SOURCES = [os.path.join(CSRC, "probes.hip")]
PROBE_HEADERS = [os.path.join(CSRC, "lattice.hpp"), os.path.join(INCLUDE, "vplbm_probes.h")]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def command(out=LIB, sources=None):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-I", INCLUDE, "-I", CSRC, "-o", out] + (sources or SOURCES)


def build(verbose: bool = False) -> str:
    _compile(LIB, SOURCES, verbose)
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return LIB


def _compile(lib, sources, verbose):
    tmp = lib + ".tmp"
    cmd = command(tmp, sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so; that line is noise.
    noise = "'-packed-fp32-ops' is not a recognized feature"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, lib)


def stale() -> bool:
    for lib, deps in ((LIB, SOURCES + HEADERS), (PROBE_LIB, PROBE_SOURCES + PROBE_HEADERS)):
        if not os.path.exists(lib):
            return True
        t = os.path.getmtime(lib)
        if any(os.path.getmtime(p) > t for p in deps):
            return True
    return False


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
