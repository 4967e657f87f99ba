"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Small cells are compared element by element on every node; the 64000- and
512000-node cells on sampled nodes computed one by one by the oracle at the
GPU's Fermi level, plus properties that hold at any size.
"""

import math
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2006_03697_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP64 path: relative to the largest magnitude of each quantity.
TOL64 = 1e-10
# Mixed path: stress in Ha/Bohr^3 (absolute).
TOL_MIXED_SIGMA = 1e-6


def _log(*a):
    print(*a, file=sys.stderr, flush=True)
    os.makedirs("gpurun_out", exist_ok=True)
    with open(os.path.join("gpurun_out", "parity_report.txt"), "a") as f:
        print(*a, file=f)


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
               moments=float(np.max(np.abs(mom - ref["moments"]))),
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


def _sampled(sq, cell, precision, nodes, name):
    """Full GPU run; the oracle on sampled nodes at the GPU's Fermi level."""
    import time
    _log("case %s precision=%s (%d sampled nodes)" % (name, precision, len(nodes)))
    t0 = time.time()
    with sq.Plan([cell], precision=precision) as P:
        rho, mu = P.density(0)
        e = P.energy(0)
        sig, parts = P.stress(0)
        rec = P.nodes(0, nodes)
        mom = P.moments(0, nodes)
        lo, hi = P.bounds(0)
    _log("  gpu run %.1fs  mu %.15g  E %.12g  sigma %s" % (time.time() - t0, mu[0], e[0],
                                                        np.array2string(sig[0], precision=8)))
    t0 = time.time()
    ref = O.run(cell, nodes=nodes, mu=float(mu[0]))
    _log("  oracle %.1fs on %d nodes" % (time.time() - t0, len(nodes)))
    err = dict(lam_lo=rel(lo[nodes], ref["lam_lo"]), lam_hi=rel(hi[nodes], ref["lam_hi"]),
               moments=float(np.max(np.abs(mom - ref["moments"]))),
               n_count=abs(np.sum(rho[0]) * cell["h"] ** 3 - cell["n_electrons"]) / cell["n_electrons"])
    err.update(_records_rel(rec, ref["records"]))
    _log("  errors", {k: "%.2e" % v for k, v in err.items()})
    return err, rec, ref


def test_64000_node_cell_fp64_sampled(sq):
    cell = W.fp64_cell()
    nodes = W.node_sample(64000, 12, seed=41)
    err, rec, ref = _sampled(sq, cell, "fp64", nodes, "40^3 nodes, 21^3 cube, npl 60")
    assert err["lam_lo"] < TOL64 and err["lam_hi"] < TOL64
    assert err["moments"] < TOL64
    assert err["n_count"] < 1e-12
    for k in ("rho_q", "e_q", "K", "N", "e_nl_q", "vrho_q", "xc_q"):
        assert err[k] < TOL64, (k, err[k])


def test_64000_node_cell_mixed_sampled(sq):
    cell = W.fp64_cell()
    nodes = W.node_sample(64000, 8, seed=42)
    err, rec, ref = _sampled(sq, cell, "mixed", nodes, "40^3 nodes, 21^3 cube, npl 60")
    assert err["n_count"] < 1e-10
    assert err["rho_q"] < 1e-2


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
    # the same computation in one batched plan or alone: they differ only by
    # the arrival order of the LDS-atomic projection sums (as repeated runs do)
    tol = 0.1 * TOL64
    for i, c in enumerate(cells):
        with sq.Plan([c], precision="fp64") as P1:
            rho1, mu1 = P1.density(0)
            e1 = P1.energy(0)
            sig1, _ = P1.stress(0)
        _log("  cell %d batched vs alone: mu %.2e rho %.2e E %.2e sigma %.2e" % (
            i, abs(mu_b[i] - mu1[0]), rel(rho_b[i], rho1[0]), abs(e_b[i] - e1[0]) / abs(e1[0]),
            rel(sig_b[i], sig1[0])))
        assert abs(mu_b[i] - mu1[0]) <= tol * max(1, abs(mu1[0]))
        assert rel(rho_b[i], rho1[0]) < tol
        assert abs(e_b[i] - e1[0]) <= tol * abs(e1[0])
        assert rel(sig_b[i], sig1[0]) < tol
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


def test_repeat_runs_agree(sq):
    # projections are summed with LDS atomics in arrival order: repeated runs
    # agree to rounding (amplified by the recurrence), not bit for bit; the
    # run-to-run spread must stay an order below the parity tolerance
    with sq.Plan([W.tiny_cell()], precision="fp64") as P:
        r1, m1 = P.density(0)
        s1, _ = P.stress(0)
        r2, m2 = P.density(0)
        s2, _ = P.stress(0)
    _log("repeat runs: mu %.2e rho %.2e sigma %.2e" % (
        abs(m1[0] - m2[0]), rel(r1[0], r2[0]), rel(s1[0], s2[0])))
    assert abs(m1[0] - m2[0]) <= 0.1 * TOL64 * max(1.0, abs(m1[0]))
    assert rel(r1[0], r2[0]) < 0.1 * TOL64
    assert rel(s1[0], s2[0]) < 0.1 * TOL64


@pytest.mark.parametrize("npl", [40, 60, 80])
def test_mixed_precision_degree_sweep(sq, npl):
    # 64000-node cell with the Chebyshev degree swept: the mixed path (FP32
    # recurrence, FP64 accumulation) against the FP64 path, which is itself
    # checked against the oracle on sampled nodes
    cell = W.fp64_cell(npl=npl)
    _log("case degree sweep npl=%d (40^3 nodes, 21^3 cube)" % npl)
    out = {}
    for prec in ("fp64", "mixed"):
        with sq.Plan([cell], precision=prec) as P:
            rho, mu = P.density(0)
            e = P.energy(0)
            sig, parts = P.stress(0)
            rec = P.nodes(0, W.node_sample(64000, 4, seed=43)) if prec == "fp64" else None
        out[prec] = dict(rho=rho[0], mu=mu[0], e=e[0], sig=sig[0], rec=rec)
    f, m = out["fp64"], out["mixed"]
    ref = O.run(cell, nodes=W.node_sample(64000, 4, seed=43), mu=float(f["mu"]))
    err64 = _records_rel(f["rec"], ref["records"])
    errs = dict(mu=abs(m["mu"] - f["mu"]), rho_max=rel(m["rho"], f["rho"]),
                rho_rms=float(np.sqrt(np.mean((m["rho"] - f["rho"]) ** 2)) / np.max(np.abs(f["rho"]))),
                e_band=abs(m["e"] - f["e"]) / abs(f["e"]),
                sigma_abs=[float(x) for x in np.abs(m["sig"] - f["sig"])])
    _log("  fp64 vs oracle (4 nodes)", {k: "%.2e" % v for k, v in err64.items()})
    _log("  mixed vs fp64: mu %.2e rho max %.2e rms %.2e E %.2e sigma %s" % (
        errs["mu"], errs["rho_max"], errs["rho_rms"], errs["e_band"],
        " ".join("%.2e" % x for x in errs["sigma_abs"])))
    for k, v in err64.items():
        assert v < TOL64, (k, v)
    assert max(errs["sigma_abs"]) < TOL_MIXED_SIGMA
    assert errs["rho_max"] < 1e-2 and errs["e_band"] < 1e-3


def test_batched_32_uneven_cells_mixed_and_fp64(sq):
    # the 32-cell stream (8-64 atoms, 10-16 Bohr, R_cut 3-4, degree 30-80,
    # kT 0.03-0.2) in one plan per precision; the densest cell needs the
    # 48-slot variant
    cells = W.batched_cells(n_cells=32, seed=3)
    _log("case batched 32 cells, %d nodes" % sum(round(c["L"][0] / c["h"]) ** 3 for c in cells))
    res = {}
    for prec in ("fp64", "mixed", "mixed_stress"):
        import time
        t0 = time.time()
        with sq.Plan(cells, precision=prec) as P:
            rho, mu = P.density(-1)
            e = P.energy(-1)
            sig, parts = P.stress(-1)
            recs = {ci: P.nodes(ci, W.node_sample(round(cells[ci]["L"][0] / cells[ci]["h"]) ** 3, 3, seed=44))
                    for ci in (0, 5)} if prec == "fp64" else None
        res[prec] = dict(rho=rho, mu=mu, e=e, sig=sig, recs=recs)
        _log("  %s: %.1f s" % (prec, time.time() - t0))
    worst = {"mixed": 0.0, "mixed_stress": 0.0}
    for i in range(len(cells)):
        d = {k: float(np.max(np.abs(res[k]["sig"][i] - res["fp64"]["sig"][i]))) for k in worst}
        for k in worst:
            worst[k] = max(worst[k], d[k])
        _log("  cell %2d: |sigma| %.3e  mixed-fp64 %.2e (mu %.2e)  mixed_stress-fp64 %.2e (mu %.2e)"
             "  npl %d kT %.3f atoms %d n %d" % (
                 i, float(np.max(np.abs(res["fp64"]["sig"][i]))), d["mixed"],
                 abs(res["mixed"]["mu"][i] - res["fp64"]["mu"][i]), d["mixed_stress"],
                 abs(res["mixed_stress"]["mu"][i] - res["fp64"]["mu"][i]), cells[i]["npl"],
                 cells[i]["kT"], len(cells[i]["pos"]), round(cells[i]["L"][0] / cells[i]["h"])))
    _log("  worst sigma abs: mixed %.2e  mixed_stress %.2e" % (worst["mixed"], worst["mixed_stress"]))
    # FP64 moments: mu as in FP64, the FP32 stress pass within the target
    assert worst["mixed_stress"] < TOL_MIXED_SIGMA
    # FP32 moments: in a cell with few states at the Fermi level (15 atoms,
    # kT 0.047) the moments' FP32 error moves mu by ~5e-6 Ha and sigma by
    # ~2.5e-6; the bound guards against regressions beyond that
    assert worst["mixed"] < 5 * TOL_MIXED_SIGMA
    for ci in (0, 5):
        c = cells[ci]
        nodes = W.node_sample(round(c["L"][0] / c["h"]) ** 3, 3, seed=44)
        ref = O.run(c, nodes=nodes, mu=float(res["fp64"]["mu"][ci]))
        err = _records_rel(res["fp64"]["recs"][ci], ref["records"])
        _log("  cell %d fp64 vs oracle" % ci, {k: "%.2e" % v for k, v in err.items()})
        for k, v in err.items():
            assert v < TOL64, (ci, k, v)


def test_512000_node_cell_mixed_vs_fp64(sq):
    # 80^3 nodes, 25^3 cubes, degree 80, 512 atoms: the mixed path against
    # the FP64 path; the FP64 path against the oracle on sampled nodes at
    # its Fermi level
    import time
    cell = W.large_cell()
    _log("case 512000-node cell (80^3 nodes, 25^3 cube, npl 80)")
    out = {}
    nodes = W.node_sample(512000, 4, seed=45)
    for prec in ("fp64", "mixed"):
        t0 = time.time()
        with sq.Plan([cell], precision=prec) as P:
            rho, mu = P.density(0)
            e = P.energy(0)
            sig, parts = P.stress(0)
            rec = P.nodes(0, nodes)
        out[prec] = dict(rho=rho[0], mu=mu[0], e=e[0], sig=sig[0], rec=rec)
        _log("  %s: %.1f s  mu %.12f  sigma %s" % (prec, time.time() - t0, mu[0],
                                                   np.array2string(sig[0], precision=8)))
    ref = O.run(cell, nodes=nodes, mu=float(out["fp64"]["mu"]))
    err = _records_rel(out["fp64"]["rec"], ref["records"])
    _log("  fp64 vs oracle (4 nodes)", {k: "%.2e" % v for k, v in err.items()})
    for k, v in err.items():
        assert v < TOL64, (k, v)
    ds = float(np.max(np.abs(out["mixed"]["sig"] - out["fp64"]["sig"])))
    _log("  mixed vs fp64: sigma abs %.2e  rho %.2e  E %.2e" % (
        ds, rel(out["mixed"]["rho"], out["fp64"]["rho"]),
        abs(out["mixed"]["e"] - out["fp64"]["e"]) / abs(out["fp64"]["e"])))
    assert ds < TOL_MIXED_SIGMA
