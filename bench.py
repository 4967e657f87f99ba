#!/usr/bin/env python3
"""SQ node-columns/s including stress, FP64 and mixed precision, on one MI355X.

A step is one pass of the whole hot path over one cell already resident in
HBM: spectral bounds (FP64 Lanczos), Chebyshev moments, Fermi level,
Clenshaw-Curtis coefficients and density (sq_density), band energy
(sq_energy), the kinetic + nonlocal stress pass (sq_stress), the direct
and trace pressures from its sums (sq_pressure) and the LDA
exchange-correlation stress term (sq_xc).  The plan
(grid, atom images, local potential, capacity census) is built before the
timed region.  Default workload: the 64000-node cell (16 Bohr cube, h = 0.4,
64 atoms, 21^3 cubes, degree 60, kT = 0.05 Ha).

Prints one JSON line.  value = node-columns/s of the FP64 path; the mixed
path (FP32 recurrence vectors, FP64 accumulation) is reported beside it.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SQ node-columns/sec incl. stress, FP64 vs mixed precision; % HBM roofline"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x FMA (2 flop) x 2.4 GHz.  FP64 vector
# FMAs and unpacked FP32 FMAs issue at the same rate (packed FP32 is not used).
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBPS = 8000.0
# LDS: 128 B per clock per CU
PEAK_LDS_TBPS = 256 * 128 * 2.4e9 / 1e12

# Algorithmic FLOPs of one application of the scaled nodal operator, per cube
# node: 37-point 12th-order stencil (37 multiply-adds), local potential
# (1 multiply-add), scale and previous-vector subtraction (2 flops); per
# (node, projector) pair: projection and projector term (2 multiply-adds).
F_POINT = 2 * 37 + 2 + 2
F_PAIR = 4


def kernel_flops(info, K, stress_fp64=True):
    """Algorithmic FLOPs of the three recurrence kernels for one cell.  The
    FP64 stress pass forms d_q by Clenshaw's recurrence (no per-step
    accumulation); with FP32 vectors it accumulates d_q += c_j t^j in FP64
    (2 FLOP per point and step)."""
    Nd, nc, npl, pairs = int(info[0]), int(info[1]), int(info[2]), int(info[8])
    pts = Nd * nc ** 3
    return {
        "lanczos": K * ((F_POINT + 8) * pts + F_PAIR * pairs),
        "moments": ((npl + 1) // 2) * ((F_POINT + 4) * pts + F_PAIR * pairs),
        "stress": npl * ((F_POINT + (0 if stress_fp64 else 2)) * pts + F_PAIR * pairs),
    }


def lds_bytes(info, K, word):
    """Algorithmic LDS bytes of the three recurrence kernels for one cell:
    the 24 in-plane stencil neighbours of every cube point read from the
    mirror and the point written back, per operator application (word =
    bytes per vector element)."""
    Nd, nc, npl = int(info[0]), int(info[1]), int(info[2])
    per = Nd * nc ** 3 * 25 * word
    return {"lanczos": K * per, "moments": ((npl + 1) // 2) * per, "stress": npl * per}


def hbm_bytes(info, K):
    """Algorithmic HBM traffic of one step (bytes): the local potential read
    by every node's cube (once per kernel pass, L2-resident in practice is
    not assumed), moments written and read, coefficients, records."""
    Nd, nc, npl = int(info[0]), int(info[1]), int(info[2])
    v = 8 * Nd * 3                     # potential column reads (three passes), per node column
    mom = 8 * Nd * (npl + 1) * 2       # moments written, read by coefficients
    coef = 8 * Nd * (npl + 1) * 2      # coefficients written, read by the stress pass
    lan = 8 * Nd * 2 * K               # Lanczos tridiagonals
    rec = 8 * Nd * 24                  # per-node records
    return v + mom + coef + lan + rec


KERNEL_SOURCES = ("paper_2006_03697_amd/csrc/sq_recur.hip", "paper_2006_03697_amd/csrc/sq_devfn.h",
                  "paper_2006_03697_amd/csrc/sq_dev.h")


def kernel_source_hash():
    """SHA-1 over the recurrence-kernel sources (identifies the build whose
    counters a profile summary records)."""
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(phase, precision, workload="64000-node cell, 21^3 cubes, degree 60"):
    """HBM bytes per launch of a kernel from the profile summaries (a line
    'traffic-json: {...}' with the counters of rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE, scaled by the same counters on a plain copy), if they were
    taken on the current kernel sources; else None."""
    import glob
    want = kernel_source_hash()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if line.startswith("traffic-json:"):
                try:
                    rec = json.loads(line.split(":", 1)[1])
                except ValueError:
                    continue
                if rec.get("phase") == phase and rec.get("precision") == precision and \
                        rec.get("workload") == workload and rec.get("source_sha1") == want:
                    return float(rec["bytes_per_launch"])
    return None


def run_precision(sq, cell, precision, steps, warmup):
    import torch
    t0 = time.time()
    plan = sq.Plan([cell], precision=precision)
    setup_s = time.time() - t0
    info = plan.info[0]

    def step():
        plan.density_only(0)
        plan.energy(0)
        plan.stress(0)
        plan.pressure(0)
        plan.xc(0)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.phase_times(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph = plan.phase_times(reset=True)
    _, mu = plan.density(0)
    sig, _ = plan.stress(0)
    pd, pt = plan.pressure(0)
    plan.close()
    ms = (t1 - t0) * 1000.0 / steps
    return dict(ms=ms, setup_s=setup_s, info=info, phases=ph, mu=float(mu[0]),
                sigma=[float(x) for x in sig[0]], p_direct=float(pd[0]), p_trace=float(pt[0]))


def cpu_baseline(cell, mu, sample):
    """The oracle as it stands, on a bounded sample of the cell's nodes at the
    GPU's Fermi level: bounds, moments, coefficients, stress pass."""
    from oracle import oracle as O
    from paper_2006_03697_amd import workloads as W
    n = int(round(cell["L"][0] / cell["h"]) * round(cell["L"][1] / cell["h"]) *
            round(cell["L"][2] / cell["h"]))
    nodes = W.node_sample(n, sample, seed=7)
    O.run(cell, nodes=nodes[:4], mu=mu)           # build + load the C core
    t0 = time.perf_counter()
    O.run(cell, nodes=nodes, mu=mu)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return dict(value=len(nodes) / dt, unit="node-columns/s", cores=cores, kind="oracle",
                sample="%d of %d nodes of the same cell (seed 7), full per-node path at the "
                       "GPU's Fermi level, %.1f s" % (len(nodes), n, dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=8192,
                    help="nodes in the oracle's CPU-baseline sample (0: skip)")
    ap.add_argument("--precision", choices=["both", "fp64", "mixed", "mixed_stress"], default="both",
                    help="both: fp64 (the headline value), mixed and mixed_stress beside it")
    ap.add_argument("--npl", type=int, default=60,
                    help="Chebyshev degree of the 64000-node cell (60; the mixed-precision "
                         "sweep of the same cell uses 40 and 80 as well)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 times) and exit: "
                         "the reference for scaling the HBM byte counters of a profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; a multi-GPU run (%d) is not part of it"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_probe > 0:
        import torch
        n = args.copy_probe * (1 << 20)
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n, "copies": 3}), flush=True)
        return

    from paper_2006_03697_amd import sq
    from paper_2006_03697_amd import workloads as W
    sq.load()
    cell = W.fp64_cell(npl=args.npl)
    K = int(cell["lanczos_steps"])
    res = {}
    for prec in (["fp64", "mixed", "mixed_stress"] if args.precision == "both" else [args.precision]):
        res[prec] = run_precision(sq, cell, prec, args.steps, args.warmup)
        print("bench: %s %.2f ms/step  phases %s" % (
            prec, res[prec]["ms"], {k: round(v[0] / max(v[1], 1), 3) for k, v in res[prec]["phases"].items()}),
            file=sys.stderr, flush=True)

    head = "fp64" if "fp64" in res else next(iter(res))
    r = res[head]
    info = r["info"]
    Nd = int(info[0])
    flops = kernel_flops(info, K, stress_fp64=head == "fp64")
    per_launch = {k: r["phases"][k][0] / max(r["phases"][k][1], 1) for k in flops}
    dom = max(per_launch, key=lambda k: per_launch[k])
    achieved = flops[dom] / (per_launch[dom] * 1e-3) / 1e12
    step_bytes = hbm_bytes(info, K)
    # bytes per vector element of the dominant kernel in the head precision
    word = 8 if head == "fp64" or (head == "mixed_stress" and dom != "stress") else 4
    lds_tbps = lds_bytes(info, K, word)[dom] / (per_launch[dom] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": Nd / (r["ms"] * 1e-3),
        "unit": "node-columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "periodic 16 Bohr cube, h 0.4 (40^3 = 64000 nodes), 64 atoms "
                               "(seed 1, min spacing 1.5), R_cut 4 (21^3 cubes), degree %d, "
                               "kT 0.05 Ha, 12th-order FD, Lanczos K=%d" % (int(info[2]), K),
                   "nodes": Nd, "cube": int(info[1]) ** 3, "npl": int(info[2]),
                   "precision": head},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved,
                     "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_VALU_TFLOPS,
                     "traffic": recorded_traffic(dom, head, "64000-node cell, 21^3 cubes, degree %d"
                                                 % int(info[2]))},
        "lds": {"kernel": dom, "achieved": lds_tbps, "peak": PEAK_LDS_TBPS, "unit": "TB/s",
                "frac": lds_tbps / PEAK_LDS_TBPS},
        "hbm": {"achieved": step_bytes / (r["ms"] * 1e-3) / 1e9, "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": step_bytes / (r["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBPS},
        "phases_ms": {k: v[0] / max(v[1], 1) for k, v in r["phases"].items()},
        "setup_s": r["setup_s"],
        "pressure": {"direct": r["p_direct"], "trace": r["p_trace"], "unit": "Ha/Bohr^3"},
    }
    for mk in ("mixed", "mixed_stress"):
        if mk not in res or head != "fp64":
            continue
        m = res[mk]
        mf = kernel_flops(m["info"], K, stress_fp64=False)
        mpl = {k: m["phases"][k][0] / max(m["phases"][k][1], 1) for k in mf}
        out[mk] = {"value": Nd / (m["ms"] * 1e-3), "ms_per_step": m["ms"], "dtype": "f32+f64",
                   "vectors": "f32 both passes" if mk == "mixed" else "f64 moments, f32 stress pass",
                   "speedup_vs_fp64": r["ms"] / m["ms"],
                   "phases_ms": {k: v[0] / max(v[1], 1) for k, v in m["phases"].items()},
                   "stress_tflops": mf["stress"] / (mpl["stress"] * 1e-3) / 1e12,
                   "mu_diff_vs_fp64": abs(m["mu"] - r["mu"]),
                   "sigma_diff_vs_fp64": max(abs(a - b) for a, b in zip(m["sigma"], r["sigma"])),
                   "p_direct_diff_vs_fp64": abs(m["p_direct"] - r["p_direct"])}
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(cell, r["mu"], args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
