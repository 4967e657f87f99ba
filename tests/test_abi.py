"""C-ABI library: it loads, exports every entry point include/sq.h declares,
and rejects invalid cells before touching the device (CPU only)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2006_03697_amd import sq
from paper_2006_03697_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    """Function names declared in every header under include/."""
    names = set()
    for f in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(sq_[a-z_0-9]+)\s*\(", text))
    return names


def test_header_declarations_match_the_binding_and_the_library():
    declared = _declared()
    assert declared == set(sq.EXPORTS)
    lib = sq.load()
    for name in declared:
        assert hasattr(lib, name), name


def _setup_status(cell):
    L = sq.load()
    keep = []
    arr = (sq.SqCell * 1)()
    arr[0] = sq._cell_struct(cell, keep)
    opt = sq.SqOptions()
    opt.precision = sq.SQ_FP64
    h = ctypes.c_void_p()
    st = L.sq_setup(arr, 1, ctypes.byref(opt), ctypes.byref(h))
    return st, L.sq_last_error(None).decode(), h


@pytest.mark.parametrize("mutate, needle", [
    (lambda c: c.update(L=(6.1, 6.0, 6.0)), "L/h"),
    (lambda c: c.update(rcut=0.3), "R_cut"),
    (lambda c: c.update(rcut=6.5), "cube width"),
    (lambda c: c.update(npl=0), "npl"),
    (lambda c: c.update(npl=300), "npl"),
    (lambda c: c.update(kT=0.0), "kT"),
    (lambda c: c.update(fd_half_order=4), "12th-order"),
    (lambda c: c.update(lanczos_steps=1), "lanczos"),
    (lambda c: c.update(species=np.array([0, 3], dtype=np.int32)), "species index"),
    (lambda c: c.update(n_electrons=1e9), "N_e"),
])
def test_setup_rejects_invalid_cells(mutate, needle):
    cell = W.tiny_cell()
    mutate(cell)
    st, msg, h = _setup_status(cell)
    assert st == sq.SQ_E_ARG
    assert needle in msg
    assert not h.value


def test_status_strings():
    L = sq.load()
    assert L.sq_status_str(sq.SQ_OK) == b"ok"
    assert L.sq_status_str(sq.SQ_E_STATE) == b"call order violated"


def test_per_width_launchers_have_internal_linkage():
    # Each cube width is a separate compile unit with launch templates of the
    # same names; an externally visible (weak) instantiation would be merged
    # across units by the linker and every width would run one width's kernels.
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-C", sq.LIB_PATH], stdout=subprocess.PIPE, text=True,
                         check=True).stdout
    bad = [ln for ln in out.splitlines()
           if re.search(r"\s[WVTu]\s", ln) and re.search(r"launch_(fp|var)", ln)]
    assert not bad, bad[:5]
    for n in (7, 9, 11, 13, 15, 17, 19, 21, 23, 25):
        for fam in ("lanczos", "moments", "stress", "gram", "census"):
            assert re.search(r"\sT sq_launch_%s_%d\(" % (fam, n), out), (fam, n)


def test_binding_fails_loudly_without_the_library():
    # no CPU fallback: a missing library is an error at load time
    import subprocess
    import sys
    code = ("import os, sys; sys.path.insert(0, %r); "
            "from paper_2006_03697_amd import sq\n"
            "try:\n    sq.load()\nexcept RuntimeError as e:\n    print('raised', e)\n") % ROOT
    env = dict(os.environ, SQ_LIB_PATH="/nonexistent/libsq_mi355x.so")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=120)
    assert "raised" in out.stdout and "missing" in out.stdout


def test_bench_algorithmic_counts():
    import sys
    sys.path.insert(0, ROOT)
    import bench
    info = [64000, 21, 60, 0, 0, 0, 0, 0, 1000, 20, 5000, 64000, 20, 0]
    pts = 64000 * 21 ** 3
    f = bench.kernel_flops(info)
    assert f["stress"] == 60 * (78 * pts + 4 * 1000)
    assert bench.kernel_flops(info, stress_fp64=False)["stress"] == 60 * (80 * pts + 4 * 1000)
    assert f["moments"] == 30 * (82 * pts + 4 * 1000)
    assert f["lanczos"] == 20 * (86 * pts + 4 * 1000)
    assert bench.lds_bytes(info, 8)["stress"] == 60 * pts * 25 * 8
    per, step = bench.hbm_bytes(info)
    # the stress pass reads the coefficients, bounds, Gram entries (12 bytes
    # each) and potential once, and writes 19 record columns
    assert per["stress"] == 8 * 64000 * 61 + 32 * 64000 + 8 * 64000 * 19 + 12 * 5000 + 8 * 64000
    # every Fermi-level evaluation re-reads the moments
    assert step > bench.MU_EVALS * 8 * 64000 * 61
    # moments from the Lanczos tridiagonal: 30 Lanczos steps, no moments pass
    quad = info[:12] + [30, 1]
    fq = bench.kernel_flops(quad)
    assert fq["lanczos"] == 30 * (86 * pts + 4 * 1000)
    assert fq["moments"] == 64000 * 60 * 7 * 31
    assert bench.lds_bytes(quad, 8)["moments"] == 0
    # a traffic record is used only for the kernel sources it was taken on
    assert bench.recorded_traffic("stress", "fp64", "no such workload") is None
    # measured HBM rate: recorded bytes per launch over the launch time
    assert bench.measured_hbm(None, 100.0) is None
    m = bench.measured_hbm(8e9, 1000.0)
    assert abs(m["achieved"] - 8.0) < 1e-12 and abs(m["frac"] - 1e-3) < 1e-15
