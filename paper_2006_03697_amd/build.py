"""Build the HIP C-ABI library for gfx950 in-tree (hipcc, no JIT cache)."""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsq_mi355x.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
EXTRA = os.environ.get("SQ_EXTRA_FLAGS", "").split()
# packed FP32 ops stay off: some of their forms have given wrong results
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

NC_LIST = [7, 9, 11, 13, 15, 17, 19, 21, 23, 25]
# (source, device code?, extra defines, object name)
UNITS = [("sq_kernels.hip", True, [], "sq_kernels_misc.o"), ("sq_capi.cpp", False, [], "sq_capi.o")] + \
        [("sq_kernels.hip", True, ["-DSQ_ONE_NC=%d" % n], "sq_kernels_nc%d.o" % n) for n in NC_LIST]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build(verbose: bool = False, jobs: int = 0, lib: str = LIB, build_dir: str = BUILD) -> str:
    """Compile every unit (per cube width in parallel) and link the library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(build_dir, exist_ok=True)
    t0 = time.time()

    def one(unit):
        src, dev, defs, objname = unit
        obj = os.path.join(build_dir, objname)
        cmd = [HIPCC] + COMMON + EXTRA + defs + (DEVICE + ["-x", "hip"] if dev else ["-ffp-contract=off"]) + \
              ["-c", os.path.join(CSRC, src), "-o", obj]
        _run(cmd)
        return obj

    jobs = jobs or min(len(UNITS), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, UNITS))
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, lib)
    if verbose:
        print("built %s in %.1fs" % (lib, time.time() - t0))
    return lib


if __name__ == "__main__":
    build(verbose=True)
