"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Small cells, compared element by element on every node; batching, bitwise
run-to-run determinism, graph replay, the persistent launch form and the
autotuner.  The 64000- and 512000-node cells and the 32-cell batch are in
test_gpu_scale.py.
"""

import math

import numpy as np
import pytest

from _gpucheck import moments_excess, report
from oracle import oracle as O
from paper_2006_03697_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP64 path: relative to the largest magnitude of each quantity.
TOL64 = 1e-10
# Mixed path: stress in Ha/Bohr^3 (absolute).
TOL_MIXED_SIGMA = 1e-6


def _log(*a):
    report(*a)


@pytest.fixture(scope="module")
def sq():
    import torch
    from paper_2006_03697_amd import sq as sqmod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sqmod.load()   # raises if the HIP library is missing
    return sqmod


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / scale) if scale > 0 else float(np.max(np.abs(a - b)))


def _records_rel(gpu, ora):
    """Per-field relative errors of [rho, e, K(9), N(9), e_nl, dV V rho]
    record blocks."""
    out = {}
    out["rho_q"] = rel(gpu[:, 0], ora[:, 0])
    out["e_q"] = rel(gpu[:, 1], ora[:, 1])
    out["K"] = rel(gpu[:, 2:11], ora[:, 2:11])
    out["N"] = rel(gpu[:, 11:20], ora[:, 11:20])
    if ora.shape[1] > 20:
        out["e_nl_q"] = rel(gpu[:, 20], ora[:, 20])
        out["vrho_q"] = rel(gpu[:, 21], ora[:, 21])
    if ora.shape[1] > 22:
        out["xc_q"] = rel(gpu[:, 22:24], ora[:, 22:24])
    return out


def _full_compare(sq, cell, precision, name):
    _log("case %s precision=%s" % (name, precision))
    ref = O.run(cell)
    with sq.Plan([cell], precision=precision) as P:
        rho, mu = P.density(0)
        e = P.energy(0)
        sig, parts = P.stress(0)
        pd, pt = P.pressure(0)
        exc, sxc = P.xc(0)
        rec = P.nodes(0, range(P.n_nodes(0)))
        lo, hi = P.bounds(0)
        mom = P.moments(0, range(P.n_nodes(0)))
    err = dict(mu=abs(mu[0] - ref["mu"]) / max(1.0, abs(ref["mu"])),
               lam_lo=rel(lo, ref["lam_lo"]), lam_hi=rel(hi, ref["lam_hi"]),
               moments=moments_excess(mom, lo, hi, ref),
               rho=rel(rho[0], ref["rho"]), e_band=abs(e[0] - ref["e_band"]) / abs(ref["e_band"]),
               sigma=rel(sig[0], ref["sigma_voigt"]),
               sigma_abs=float(np.max(np.abs(sig[0] - ref["sigma_voigt"]))),
               K=rel(parts[0][:9], ref["parts"][:9]), N=rel(parts[0][9:], ref["parts"][9:]),
               p_direct=abs(pd[0] - ref["pressure_direct"]) / abs(ref["pressure_direct"]),
               p_trace=abs(pt[0] - ref["pressure_trace"]) / abs(ref["pressure_trace"]),
               p_abs=max(abs(pd[0] - ref["pressure_direct"]), abs(pt[0] - ref["pressure_trace"])),
               e_xc=abs(exc[0] - ref["e_xc"]) / abs(ref["e_xc"]),
               sigma_xc=abs(sxc[0] - ref["sigma_xc"]) / abs(ref["sigma_xc"]))
    err.update({"rec_" + k: v for k, v in _records_rel(rec, ref["records"]).items()})
    _log("  errors", {k: "%.2e" % v for k, v in err.items()})
    _log("  mu gpu %.15g oracle %.15g; sigma gpu %s oracle %s" % (
        mu[0], ref["mu"], np.array2string(sig[0], precision=10),
        np.array2string(ref["sigma_voigt"], precision=10)))
    _log("  pressure gpu direct %.15g trace %.15g; oracle direct %.15g trace %.15g" % (
        pd[0], pt[0], ref["pressure_direct"], ref["pressure_trace"]))
    return err, ref, dict(rho=rho[0], mu=mu[0], e=e[0], sig=sig[0], parts=parts[0], rec=rec,
                          p_direct=pd[0], p_trace=pt[0])


def test_tiny_cell_fp64_every_node(sq):
    err, ref, g = _full_compare(sq, W.tiny_cell(), "fp64", "tiny 12^3 nodes, 9^3 cube")
    # intermediate quantities: FP64 rounding differences (FMA, reduction
    # order, the doubling identities) stay far below the output tolerance
    assert err["lam_lo"] < TOL64 and err["lam_hi"] < TOL64
    assert err["moments"] < TOL64
    assert err["mu"] < TOL64
    for k in ("rho", "e_band", "sigma", "K", "N", "rec_rho_q", "rec_e_q", "rec_K", "rec_N",
              "rec_e_nl_q", "rec_vrho_q", "rec_xc_q", "p_direct", "p_trace", "e_xc", "sigma_xc"):
        assert err[k] < TOL64, (k, err[k])


def test_tiny_cell_mixed(sq):
    err, ref, g = _full_compare(sq, W.tiny_cell(), "mixed", "tiny 12^3 nodes, 9^3 cube")
    assert err["sigma_abs"] < TOL_MIXED_SIGMA
    assert err["p_abs"] < TOL_MIXED_SIGMA
    assert err["rho"] < 1e-3 and err["e_band"] < 1e-4


def test_tiny_cell_mixed_stress(sq):
    err, ref, g = _full_compare(sq, W.tiny_cell(), "mixed_stress", "tiny 12^3 nodes, 9^3 cube")
    # FP64 moments: Fermi level, density and band energy as in FP64
    assert err["mu"] < TOL64 and err["rho"] < TOL64 and err["e_band"] < TOL64
    assert err["sigma_abs"] < TOL_MIXED_SIGMA
    assert err["p_abs"] < TOL_MIXED_SIGMA


def test_ragged_cell_fp64_every_node(sq):
    # 17^3 nodes (ragged node tiles), 15^3 cubes, several atoms
    cell = W.random_cell(seed=11, L=6.8, h=0.4, n_atoms=6, d_min=1.5, rcut=3.0, npl=30, kT=0.1)
    err, ref, g = _full_compare(sq, cell, "fp64", "ragged 17^3 nodes, 15^3 cube")
    for k in ("rho", "e_band", "sigma", "K", "N", "rec_rho_q", "rec_K", "rec_N", "rec_e_nl_q",
              "rec_vrho_q", "rec_xc_q", "p_direct", "p_trace", "e_xc", "sigma_xc"):
        assert err[k] < TOL64, (k, err[k])
    assert abs(np.sum(g["rho"]) * cell["h"] ** 3 - cell["n_electrons"]) < 1e-11 * cell["n_electrons"]


def test_dense_cell_fp64_every_node(sq):
    # 13 atoms in a 6 Bohr cube: 900 to 1260 overlapping projector pairs per
    # cube, so some cubes keep their Gram matrix (one sweep per step) and the
    # others exceed its capacity (two sweeps per step); up to 28 images cross
    # one column
    cell = W.random_cell(seed=21, L=6.0, h=0.5, n_atoms=13, d_min=1.2, rcut=2.0, npl=24, kT=0.1)
    err, ref, g = _full_compare(sq, cell, "fp64", "dense 12^3 nodes, 13 atoms, 9^3 cube")
    for k in ("rho", "e_band", "sigma", "K", "N", "rec_rho_q", "rec_e_q", "rec_K", "rec_N",
              "rec_e_nl_q", "rec_vrho_q", "p_direct", "p_trace"):
        assert err[k] < TOL64, (k, err[k])


def test_dense_cell_mixed(sq):
    cell = W.random_cell(seed=21, L=6.0, h=0.5, n_atoms=13, d_min=1.2, rcut=2.0, npl=24, kT=0.1)
    err, ref, g = _full_compare(sq, cell, "mixed", "dense 12^3 nodes, 13 atoms, 9^3 cube")
    assert err["sigma_abs"] < TOL_MIXED_SIGMA and err["p_abs"] < TOL_MIXED_SIGMA


def test_fixed_fermi_level_mode(sq):
    cell = W.tiny_cell(npl=20)
    cell["mu_mode"] = "fixed"
    cell["mu"] = 0.3
    _log("case tiny fixed mu=0.3")
    ref = O.run(cell)
    with sq.Plan([cell], precision="fp64") as P:
        rho, mu = P.density(0)
        sig, parts = P.stress(0)
    assert mu[0] == 0.3
    assert rel(rho[0], ref["rho"]) < TOL64
    assert rel(sig[0], ref["sigma_voigt"]) < TOL64


def test_batched_uneven_cells_match_single_cell_runs(sq):
    cells = W.batched_cells(n_cells=4, seed=3)
    # shrink to keep the test short: the first four cells of the stream
    _log("case batched 4 uneven cells: " + ", ".join(
        "%d^3/%d^3 npl %d" % (round(c["L"][0] / 0.4), 2 * math.floor(c["rcut"] / 0.4 + 1e-9) + 1,
                               c["npl"]) for c in cells))
    with sq.Plan(cells, precision="fp64") as P:
        rho_b, mu_b = P.density(-1)
        e_b = P.energy(-1)
        sig_b, parts_b = P.stress(-1)
    # the same computation in one batched plan or alone: every node runs the
    # same kernel variant and every sum is formed in a fixed order, so the
    # results agree bit for bit
    for i, c in enumerate(cells):
        with sq.Plan([c], precision="fp64") as P1:
            rho1, mu1 = P1.density(0)
            e1 = P1.energy(0)
            sig1, _ = P1.stress(0)
        _log("  cell %d batched vs alone: mu %.2e rho %.2e E %.2e sigma %.2e" % (
            i, abs(mu_b[i] - mu1[0]), rel(rho_b[i], rho1[0]), abs(e_b[i] - e1[0]) / abs(e1[0]),
            rel(sig_b[i], sig1[0])))
        assert mu_b[i] == mu1[0]
        assert np.array_equal(rho_b[i], rho1[0])
        assert e_b[i] == e1[0]
        assert np.array_equal(sig_b[i], sig1[0])
    # one cell of the batch against the oracle on sampled nodes
    c = cells[0]
    n = int(round(c["L"][0] / c["h"])) ** 3
    nodes = W.node_sample(n, 6, seed=5)
    with sq.Plan([c], precision="fp64") as P1:
        rho1, mu1 = P1.density(0)
        P1.stress(0)
        rec = P1.nodes(0, nodes)
    ref = O.run(c, nodes=nodes, mu=float(mu1[0]))
    err = _records_rel(rec, ref["records"])
    _log("  batched cell 0 vs oracle", {k: "%.2e" % v for k, v in err.items()})
    for k, v in err.items():
        assert v < TOL64, (k, v)


def test_call_order_is_enforced(sq):
    with sq.Plan([W.tiny_cell()], precision="fp64") as P:
        with pytest.raises(sq.SqError) as e:
            P.energy(0)
        assert e.value.status == sq.SQ_E_STATE
        with pytest.raises(sq.SqError) as e:
            P.stress(0)
        assert e.value.status == sq.SQ_E_STATE
        with pytest.raises(sq.SqError) as e:
            P.pressure(0)
        assert e.value.status == sq.SQ_E_STATE
        with pytest.raises(sq.SqError) as e:
            P.xc(0)
        assert e.value.status == sq.SQ_E_STATE


def test_pressure_runs_the_stress_pass_when_needed(sq):
    # sq_pressure straight after sq_density runs the stress pass itself; after
    # a new sq_density the stress columns start from zero again
    cell = W.tiny_cell()
    _log("case tiny pressure without sq_stress")
    with sq.Plan([cell], precision="fp64") as P:
        P.density(0)
        pd1, pt1 = P.pressure(0)
        sig1, _ = P.stress(0)
        pd2, pt2 = P.pressure(0)
        P.density(0)
        rec = P.nodes(0, range(P.n_nodes(0)))
        pd3, pt3 = P.pressure(0)
    assert np.all(rec[:, 2:21] == 0.0) and np.all(rec[:, 21] != 0.0)
    for a, b in ((pd1, pd2), (pt1, pt2), (pd1, pd3), (pt1, pt3)):
        assert abs(a[0] - b[0]) < 0.1 * TOL64 * abs(b[0])
    # same sums in another rounding order; tr K and tr N largely cancel, so
    # the agreement is a few hundred ulps of the result, not one
    assert abs(pt1[0] + (sig1[0][0] + sig1[0][1] + sig1[0][2]) / 3) < 1e-12 * abs(pt1[0])


def _run_all(P, cell=0):
    rho, mu = P.density(cell)
    e = P.energy(cell)
    sig, parts = P.stress(cell)
    pd, pt = P.pressure(cell)
    rec = P.nodes(0, range(P.n_nodes(0)))
    return dict(rho=rho, mu=mu, e=e, sig=sig, parts=parts, pd=pd, pt=pt, rec=rec)


def _same(x, y):
    if isinstance(x, (list, tuple)):
        return len(x) == len(y) and all(_same(u, v) for u, v in zip(x, y))
    return np.array_equal(np.asarray(x), np.asarray(y))


def _bitwise(a, b):
    return all(_same(a[k], b[k]) for k in a)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_repeat_runs_are_bitwise_identical(sq, precision):
    # projections, Gram entries and near-image sums are exact integer sums
    # and every reduction has a fixed order: a repeated run reproduces every
    # bit (a race or an order-dependent sum would show here)
    cells = [W.tiny_cell(), W.tiny_cell(seed=9, n_atoms=4)]
    with sq.Plan(cells, precision=precision) as P:
        r1 = _run_all(P, -1)
        r2 = _run_all(P, -1)
    with sq.Plan(cells, precision=precision) as P:
        r3 = _run_all(P, -1)
    _log("repeat runs (%s): bitwise %s / new plan %s" % (precision, _bitwise(r1, r2), _bitwise(r1, r3)))
    assert _bitwise(r1, r2)
    assert _bitwise(r1, r3)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replays_equal_eager(sq, precision):
    # density -> energy -> stress captured in HIP graphs at the first call,
    # replayed at the next ones, with the program's own eager work and
    # synchronisations between replays: every replay equals the eager run
    import torch
    cells = [W.tiny_cell(), W.make_cell(6.0, 0.5, np.array([[1.0, 2.0, 3.0], [4.0, 4.5, 1.5]]),
                                        2.5, 31, 0.08)]
    with sq.Plan(cells, precision=precision) as P:
        ref = _run_all(P, -1)
    with sq.Plan(cells, precision=precision, use_graph=True) as P:
        for rep in range(4):
            x = torch.randn(1 << 20, device="cuda:0")
            (x * 2.0).sum().item()
            torch.cuda.synchronize()
            got = _run_all(P, -1)
            _log("graph replay %d (%s): bitwise %s" % (rep, precision, _bitwise(ref, got)))
            assert _bitwise(ref, got), rep
        # a single-cell selection has graphs of its own
        r0 = P.density(0)
        assert np.array_equal(r0[0][0], ref["rho"][0]) and r0[1][0] == ref["mu"][0]


def test_persistent_launch_equals_per_node_launch(sq):
    cells = W.batched_cells(n_cells=3, seed=11)
    with sq.Plan(cells, precision="fp64") as P:
        a = _run_all(P, -1)
    with sq.Plan(cells, precision="fp64", persistent=True) as P:
        b = _run_all(P, -1)
    with sq.Plan(cells, precision="fp64", persistent=True, use_graph=True) as P:
        _run_all(P, -1)
        c = _run_all(P, -1)
    _log("persistent vs per-node: bitwise %s, with graph %s" % (_bitwise(a, b), _bitwise(a, c)))
    assert _bitwise(a, b) and _bitwise(a, c)


def test_autotune_and_its_cache(sq, tmp_path):
    # the tuner times the variants of every node group and writes its
    # choices; a second plan with the same cache reads them back (no timing);
    # variants share the arithmetic of every step, so results do not depend
    # on the choice beyond rounding of the plane-0 projector weights
    import json
    import time
    cells = [W.tiny_cell(), W.batched_cells(n_cells=1, seed=12)[0]]
    path = str(tmp_path / "tune.json")
    with sq.Plan(cells, precision="fp64") as P:
        a = _run_all(P, -1)
    t0 = time.time()
    with sq.Plan(cells, precision="fp64", autotune=True, tune_cache=path) as P:
        t_tune = time.time() - t0
        b = _run_all(P, -1)
    with open(path) as f:
        table = json.load(f)
    assert len(table) > 0
    t0 = time.time()
    with sq.Plan(cells, precision="fp64", autotune=True, tune_cache=path) as P:
        t_hit = time.time() - t0
        c = _run_all(P, -1)
    _log("autotune: %d entries, set-up %.2f s tuning / %.2f s cached; %s" % (
        len(table), t_tune, t_hit, json.dumps(table)[:300]))
    assert _bitwise(b, c)
    for k in ("rho", "sig", "e"):
        for x, y in zip(a[k], b[k]):
            assert rel(x, y) < 1e-12, k
