"""Degenerate and extreme cases of the method on the HIP path (through the
C ABI), each checked against the FP64 CPU oracle on every node:

* a cell without atoms (uniform electron gas on the grid: no projector
  slots, no images);
* projector energy gamma = 0 (the nonlocal terms vanish identically);
* one atom sitting on a grid node of a cubic cell (the stress is isotropic);
* odd, and the smallest, Chebyshev degrees (the odd-degree branch of
  Clenshaw's recurrence, n_pl = 1 and 2);
* 7^3 cubes reached by more atom images than the workgroup has threads,
  with and without a stored Gram matrix;
* the error paths: N_e out of range, a Fermi-level search stopped at its
  update cap, spectral bounds too narrow, a device allocation that fails
  (forced from the host; every kernel exits normally).
"""

import ctypes
import math

import numpy as np
import pytest

from _gpucheck import moments_excess, report
from oracle import oracle as O
from paper_2006_03697_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _log(*a):
    report(*a)


@pytest.fixture(scope="module")
def sq():
    import torch
    from paper_2006_03697_amd import sq as sqmod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sqmod.load()
    return sqmod


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / scale) if scale > 0 else float(np.max(np.abs(a - b)))


def _every_node(sq, cell, name, precision="fp64"):
    """GPU run of every entry point and the oracle on every node; returns
    the errors and both results."""
    _log("case %s" % name)
    ref = O.run(cell)
    with sq.Plan([cell], precision=precision) as P:
        rho, mu = P.density(0)
        e = P.energy(0)
        sig, parts = P.stress(0)
        pd, pt = P.pressure(0)
        rec = P.nodes(0, range(P.n_nodes(0)))
        mom = P.moments(0, range(P.n_nodes(0)))
        lo, hi = P.bounds(0)
        info = P.info[0].copy()
    err = dict(mu=abs(mu[0] - ref["mu"]) / max(1.0, abs(ref["mu"])),
               moments=moments_excess(mom, lo, hi, ref),
               rho=rel(rho[0], ref["rho"]),
               e_band=abs(e[0] - ref["e_band"]) / max(abs(ref["e_band"]), 1e-300),
               sigma=rel(sig[0], ref["sigma_voigt"]),
               K=rel(parts[0][:9], ref["parts"][:9]),
               rec=rel(rec[:, :22], ref["records"][:, :22]),
               p_direct=abs(pd[0] - ref["pressure_direct"]) / abs(ref["pressure_direct"]))
    _log("  errors", {k: "%.2e" % v for k, v in err.items()})
    return err, ref, dict(rho=rho[0], mu=mu[0], e=e[0], sig=sig[0], parts=parts[0], rec=rec, info=info)


def _assert_all(err, skip=()):
    for k, v in err.items():
        if k not in skip:
            assert v < TOL64, (k, v)


def test_no_atoms(sq):
    # a uniform electron gas on the grid: every node's cube is the same, so
    # the density is uniform and the stress isotropic (kT 1 Ha and degree 80
    # converge the expansion over the cube's spectrum [0.6, 40.6] Ha; with a
    # Fermi level below the spectrum, e.g. 4 electrons at kT 0.1, the stress
    # would be a Boltzmann tail that rounding of the bounds moves at 1e-7)
    cell = W.make_cell(6.0, 0.5, np.zeros((0, 3)), 2.0, 80, 1.0, n_electrons=400.0)
    err, ref, g = _every_node(sq, cell, "no atoms, 12^3 nodes, 9^3 cube, n_e 400")
    _assert_all(err)
    assert g["info"][3] == 0
    rho = g["rho"]
    assert np.max(rho) - np.min(rho) <= 1e-13 * np.max(rho)
    assert abs(np.sum(rho) * 0.125 - 400.0) < 1e-12 * 400.0
    s = g["sig"]
    assert np.max(np.abs(s[3:])) <= 1e-12 * np.max(np.abs(s[:3]))
    assert np.max(np.abs(s[:3] - s[0])) <= 1e-12 * abs(s[0])
    # no projectors: the nonlocal parts and energy are exactly zero
    assert np.all(g["parts"][9:] == 0.0) and np.all(g["rec"][:, 11:21] == 0.0)


def test_zero_projector_energy(sq):
    sp = dict(W.GAUSS_SPECIES, gamma=0.0)
    cell = W.tiny_cell(species_params=[sp])
    err, ref, g = _every_node(sq, cell, "tiny cell, gamma = 0")
    _assert_all(err)
    assert np.all(g["parts"][9:] == 0.0) and np.all(g["rec"][:, 11:21] == 0.0)


def test_single_atom_on_a_node(sq):
    # one atom on grid node (6, 6, 6) of the 12^3 grid of a 6 Bohr cube: the
    # grid, the cell and the atom share the cubic point group, so sigma is a
    # multiple of the identity
    cell = W.make_cell(6.0, 0.5, np.array([[3.0, 3.0, 3.0]]), 2.0, 80, 1.0, n_electrons=60.0)
    err, ref, g = _every_node(sq, cell, "one atom on a node, 12^3 nodes, n_e 60")
    _assert_all(err)
    s = g["sig"]
    scale = np.max(np.abs(s))
    _log("  sigma", np.array2string(s, precision=14))
    assert np.max(np.abs(s[3:])) <= 1e-12 * scale
    assert np.max(np.abs(s[:3] - s[0])) <= 1e-12 * scale
    # and the off-diagonal node sums of K and of N vanish separately
    off = np.array([1, 2, 3, 5, 6, 7])
    assert np.max(np.abs(g["parts"][off])) <= 1e-12 * np.max(np.abs(g["parts"][:9]))
    assert np.max(np.abs(g["parts"][9 + off])) <= 1e-12 * np.max(np.abs(g["parts"][9:]))


@pytest.mark.parametrize("npl", [1, 2, 23])
def test_small_and_odd_degrees(sq, npl):
    cell = W.tiny_cell(npl=npl)
    err, ref, g = _every_node(sq, cell, "tiny cell, npl %d (every node)" % npl)
    _assert_all(err)


def _crowded(sq, n_atoms, p_sigma, p_rcut, seed, d_min):
    sp = dict(W.GAUSS_SPECIES, p_sigma=p_sigma, p_rcut=p_rcut)
    return W.random_cell(seed=seed, L=6.0, h=0.5, n_atoms=n_atoms, d_min=d_min, rcut=1.5, npl=24,
                         kT=0.2, species_params=[sp])


def test_crowded_7_cube_two_sweeps(sq):
    # 7^3 cubes (64 threads per workgroup) reached by ~90 projector images,
    # up to ~40 across one column: far more overlapping pairs (~1800) than
    # the stored Gram matrix holds, so every step takes two sweeps
    cell = _crowded(sq, 20, 0.6, 3.6, seed=7, d_min=1.0)
    err, ref, g = _every_node(sq, cell, "7^3 cube, 20 atoms, broad projectors")
    _log("  census images/cube %d  per column %d  pairs %d" % (g["info"][5], g["info"][6], g["info"][8]))
    assert g["info"][1] == 7 and g["info"][5] > 64
    _assert_all(err)


def test_crowded_7_cube_stored_gram(sq):
    # the same cube width reached by ~80 images, but with narrow projectors
    # (about 110 overlapping pairs, within the stored Gram matrix's 256): the
    # single-sweep form with Gram rows of images past the thread count
    cell = _crowded(sq, 250, 0.25, 0.5, seed=8, d_min=0.7)
    err, ref, g = _every_node(sq, cell, "7^3 cube, 250 atoms, narrow projectors")
    _log("  census images/cube %d  per column %d  pairs %d" % (g["info"][5], g["info"][6], g["info"][8]))
    assert g["info"][1] == 7 and g["info"][5] > 64
    _assert_all(err)


# ---------------------------------------------------------------------------
# error paths
# ---------------------------------------------------------------------------

def test_electron_count_out_of_range(sq):
    # N_e must lie in (0, 2 N_d): the grid holds at most two electrons per
    # node, so no Fermi level reaches more
    cell = W.tiny_cell()
    cell["n_electrons"] = 2.0 * 12 ** 3
    with pytest.raises(sq.SqError) as e:
        sq.Plan([cell], precision="fp64")
    assert e.value.status == sq.SQ_E_ARG


def test_fermi_search_cap(sq):
    with sq.Plan([W.tiny_cell()], precision="fp64", inject=sq.SQ_INJECT_MU_CAP) as P:
        with pytest.raises(sq.SqError) as e:
            P.density(0)
        assert e.value.status == sq.SQ_E_NOCONV
        assert "cap" in str(e.value)
        # nothing downstream runs on a failed density
        with pytest.raises(sq.SqError) as e:
            P.stress(0)
        assert e.value.status == sq.SQ_E_STATE


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bounds_too_narrow(sq, precision):
    with sq.Plan([W.tiny_cell()], precision=precision, inject=sq.SQ_INJECT_NARROW) as P:
        with pytest.raises(sq.SqError) as e:
            P.density(0)
        assert e.value.status == sq.SQ_E_BOUNDS


def test_allocation_failure(sq):
    # an allocator that fails on its fifth request: sq_setup returns
    # SQ_E_ALLOC and hands every block it got back to dev_free
    import torch
    L = sq.load()
    held = {}
    calls = {"n": 0}

    def alloc(nbytes, ctx):
        calls["n"] += 1
        if calls["n"] >= 5:
            return None
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda:0")
        held[t.data_ptr()] = t
        return t.data_ptr()

    def free(ptr, ctx):
        held.pop(ptr, None)

    a_cb, f_cb = sq.ALLOC_FN(alloc), sq.FREE_FN(free)
    keep = []
    cells = (sq.SqCell * 1)()
    cells[0] = sq._cell_struct(W.tiny_cell(), keep)
    opt = sq.SqOptions()
    opt.precision = sq.PRECISIONS["fp64"]
    opt.hip_stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    opt.dev_alloc = a_cb
    opt.dev_free = f_cb
    h = ctypes.c_void_p()
    st = L.sq_setup(cells, 1, ctypes.byref(opt), ctypes.byref(h))
    assert st == sq.SQ_E_ALLOC, st
    assert not h.value
    assert calls["n"] >= 5 and not held
    assert b"alloc" in L.sq_last_error(None).lower()
