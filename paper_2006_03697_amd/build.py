"""Build the HIP C-ABI library for gfx950 in-tree (hipcc, no JIT cache).

Units: the width-independent kernels (sq_misc.hip), the host plan
(sq_capi.cpp) and the recurrence kernels once per cube width
(sq_recur.hip with SQ_ONE_NC), compiled in parallel.  An object is rebuilt
when it is missing, older than its source or a shared header, or was built
with other flags; build(force=True) rebuilds everything.
"""
import hashlib
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
HEADERS = [os.path.join(INCLUDE, "sq.h"), os.path.join(INCLUDE, "sq_probe.h"), os.path.join(CSRC, "sq_dev.h"),
           os.path.join(CSRC, "sq_devfn.h")]

# roctx ranges over the entry points (rocprofv3 --marker-trace)
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]

NC_LIST = [7, 9, 11, 13, 15, 17, 19, 21, 23, 25]
# (source, device code?, extra defines, object name)
UNITS = [("sq_misc.hip", True, [], "sq_misc.o"), ("sq_capi.cpp", False, [], "sq_capi.o"),
         ("sq_probe.hip", True, [], "sq_probe.o")] + \
        [("sq_recur.hip", True, ["-DSQ_ONE_NC=%d" % n], "sq_recur_nc%d.o" % n) for n in NC_LIST]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def _stale(obj, src, cmd):
    stamp = obj + ".cmd"
    key = hashlib.sha1(" ".join(cmd).encode()).hexdigest()
    if not os.path.exists(obj) or not os.path.exists(stamp):
        return True, stamp, key
    if open(stamp).read().strip() != key:
        return True, stamp, key
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src] + HEADERS), stamp, key


def build(verbose: bool = False, jobs: int = 0, lib: str = LIB, build_dir: str = BUILD,
          force: bool = False, csrc: str = CSRC, units=None) -> str:
    """Compile the stale units (per cube width in parallel) and link the library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(build_dir, exist_ok=True)
    t0 = time.time()
    units = UNITS if units is None else units

    def one(unit):
        src, dev, defs, objname = unit
        obj = os.path.join(build_dir, objname)
        path = os.path.join(csrc, src)
        cmd = [HIPCC] + COMMON + EXTRA + defs + (DEVICE + ["-x", "hip"] if dev else ["-ffp-contract=off"]) + \
              ["-c", path, "-o", obj]
        stale, stamp, key = _stale(obj, path, cmd)
        if stale or force:
            _run(cmd)
            with open(stamp, "w") as f:
                f.write(key + "\n")
        return obj

    jobs = jobs or min(len(units), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, units))
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs + LINK)
    os.replace(tmp, lib)
    if verbose:
        print("built %s in %.1fs" % (lib, time.time() - t0))
    return lib


if __name__ == "__main__":
    build(verbose=True, force="--force" in sys.argv)
