#!/usr/bin/env python3
"""SQ node-columns/s including stress, FP64 and mixed precision, on one MI355X.

A step is one pass of the whole hot path over cells already resident in HBM:
spectral bounds (FP64 Lanczos), Chebyshev moments, Fermi level,
Clenshaw-Curtis coefficients and density (sq_density), band energy
(sq_energy), the kinetic + nonlocal stress pass (sq_stress), the direct and
trace pressures from its sums (sq_pressure) and the LDA exchange-correlation
stress term (sq_xc).  Each plan (grid, atom images, local potential,
capacity census, Gram matrices, autotuning) is built before the timed region;
sq_density and the stress pass are replayed from HIP graphs captured at the
first (warm-up) call.

Headline (value): the 64000-node cell (16 Bohr cube, h = 0.4, 64 atoms, 21^3
cubes, degree 60, kT = 0.05 Ha) on the FP64 path.  Beside it: the same cell
on the mixed paths, the 32-cell uneven batch (one plan, autotuned) and the
512000-node cell, each in FP64 and mixed.

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SQ node-columns/sec incl. stress, FP64 vs mixed precision; % HBM roofline"
# MI355X: 256 CUs x 4 SIMD x 16 FP64 lanes x FMA (2 flop) x 2.4 GHz
PEAK_F64_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12     # 78.6
PEAK_HBM_GBPS = 8000.0

# Algorithmic FLOPs of one application of the scaled nodal operator, per cube
# node: 37-point 12th-order stencil (37 multiply-adds), local potential
# (1 multiply-add), scale and previous-vector subtraction (2 flops); per
# (node, projector) pair: projection and projector term (2 multiply-adds).
F_POINT = 2 * 37 + 2 + 2
F_PAIR = 4
MU_EVALS = 48   # Fermi-level evaluations launched per sq_density (converged ones skip their reads)


def lanczos_run(info):
    """(Lanczos steps run per node, moments from the Lanczos tridiagonal)."""
    if len(info) > 13:
        return int(info[12]), bool(info[13])
    return int(info[9]), False


def kernel_flops(info, stress_fp64=True):
    """Algorithmic FLOPs of the recurrence kernels for one cell.  The FP64
    stress pass forms d_q by Clenshaw's recurrence (no per-step
    accumulation); with FP32 vectors it accumulates d_q += c_j t^j in FP64
    (2 FLOP per point and step).  Moments from the Lanczos tridiagonal cost
    7 FLOP per component of the (k + 1)-vector and degree."""
    Nd, nc, npl, pairs = int(info[0]), int(info[1]), int(info[2]), int(info[8])
    kr, quad = lanczos_run(info)
    pts = Nd * nc ** 3
    return {
        "lanczos": kr * ((F_POINT + 8) * pts + F_PAIR * pairs),
        "moments": (Nd * npl * 7 * (kr + 1) if quad else
                    ((npl + 1) // 2) * ((F_POINT + 4) * pts + F_PAIR * pairs)),
        "stress": npl * ((F_POINT + (0 if stress_fp64 else 2)) * pts + F_PAIR * pairs),
    }


def lds_bytes(info, word):
    """Algorithmic LDS bytes of the recurrence kernels for one cell: the 24
    in-plane stencil neighbours of every cube point read from the mirror and
    the point written back, per operator application (word = bytes per
    vector element); none for moments from the Lanczos tridiagonal."""
    Nd, nc, npl = int(info[0]), int(info[1]), int(info[2])
    kr, quad = lanczos_run(info)
    per = Nd * nc ** 3 * 25 * word
    return {"lanczos": kr * per, "moments": 0 if quad else ((npl + 1) // 2) * per, "stress": npl * per}


def hbm_bytes(info):
    """Compulsory HBM traffic (bytes), per kernel pass and per step, of one
    cell: every array read or written once per pass (re-reads within a pass
    hit the caches: the node's potential columns, its Gram entries at every
    recurrence step), except the moments, which every Fermi-level evaluation
    reads again (MU_EVALS, an upper bound: a converged search skips them)."""
    Nd, nc, npl = int(info[0]), int(info[1]), int(info[2])
    kr, quad = lanczos_run(info)
    gram = 12 * int(info[10])                      # value (8) + index pair (4)
    vloc = 8 * Nd
    lan = {"lanczos": 8 * Nd * 2 * kr + 4 * Nd + gram + vloc,
           "moments": (8 * Nd * (npl + 1) + 32 * Nd + (8 * Nd * 2 * kr + 4 * Nd if quad else gram + vloc)),
           "stress": 8 * Nd * (npl + 1) + 32 * Nd + 8 * Nd * 19 + gram + vloc}
    step = (lan["lanczos"] + lan["moments"] + lan["stress"] +
            8 * Nd * (npl + 1) * MU_EVALS +           # moments re-read by the Fermi-level search
            8 * Nd * (npl + 1) * 2 + 8 * Nd * 4 +     # coefficients written; bounds
            8 * Nd * 24)                               # records of the final reductions
    return lan, step


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


def recorded_traffic(phase, precision, workload):
    """HBM bytes per launch of a kernel from the profile summaries (a line
    'traffic-json: {...}' with rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by
    the same counters on a plain copy), if they were taken on the current
    kernel sources; else None."""
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


def measured_hbm(bytes_per_launch, launch_ms):
    """HBM rate of the dominant kernel from its recorded rocprofv3 traffic
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated) over its launch time; None
    when no record matches the current kernel sources."""
    if bytes_per_launch is None or not launch_ms:
        return None
    gbps = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    return {"bytes_per_launch": bytes_per_launch, "achieved": gbps, "frac": gbps / PEAK_HBM_GBPS,
            "kind": "rocprofv3 FETCH_SIZE + WRITE_SIZE of the dominant kernel, copy-calibrated"}


def run_plan(sq, cells, precision, steps, warmup, **plan_kw):
    """Times `steps` whole steps over every cell of one plan (after
    `warmup`); per-phase device times from the plan's HIP events."""
    import torch
    t0 = time.time()
    plan = sq.Plan(cells, precision=precision, **plan_kw)
    setup_s = time.time() - t0
    info = [i.copy() for i in plan.info]

    last = {}

    def step():
        last["mu"] = plan.density_only(-1)
        plan.energy(-1)
        last["sig"], _ = plan.stress(-1)
        last["pd"], last["pt"] = plan.pressure(-1)
        plan.xc(-1)

    label = "%d cell%s, %d nodes, %s" % (len(cells), "" if len(cells) == 1 else "s",
                                         sum(int(i[0]) for i in info), precision)
    for k in range(warmup):
        ta = time.perf_counter()
        step()
        torch.cuda.synchronize()
        print("bench:   warm-up %d (%s): %.2f s" % (k, label, time.perf_counter() - ta), file=sys.stderr, flush=True)
    plan.phase_times(reset=True)
    times = []
    for k in range(steps):
        ta = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ta)
        if steps <= 3 or times[-1] > 5.0:
            print("bench:   step %d (%s): %.2f s" % (k, label, times[-1]), file=sys.stderr, flush=True)
    ph = plan.phase_times(reset=True)
    mu, sig, pd, pt = last["mu"], last["sig"], last["pd"], last["pt"]   # of the last timed step
    plan.close()
    times.sort()
    ms = 1000.0 * times[len(times) // 2]   # median step
    nodes = sum(int(i[0]) for i in info)
    return dict(ms=ms, ms_mean=1000.0 * sum(times) / len(times), setup_s=setup_s, info=info,
                nodes=nodes, phases=ph, mu=[float(x) for x in mu], sigma=[[float(x) for x in s] for s in sig],
                p_direct=[float(x) for x in pd], p_trace=[float(x) for x in pt])


def per_launch(res):
    return {k: v[0] / max(v[1], 1) for k, v in res["phases"].items()}


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
    ap.add_argument("--precision", choices=["all", "fp64", "mixed", "mixed_stress"], default="all",
                    help="all: fp64 (the headline value), mixed and mixed_stress beside it")
    ap.add_argument("--npl", type=int, default=60, help="Chebyshev degree of the 64000-node cell")
    ap.add_argument("--extra", type=int, default=1,
                    help="1: also the 32-cell batch and the 512000-node cell (one timed step each)")
    ap.add_argument("--eager", action="store_true", help="launch eagerly instead of replaying graphs")
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
    graph = not args.eager
    # measured LDS read peaks (16-byte reads: the FP64 mirror; 8-byte: FP32)
    lds_peak = {w: sq.probe_lds(w) for w in (16, 8)}
    print("bench: LDS peak %s" % {w: "%.1f TB/s" % v[0] for w, v in lds_peak.items()}, file=sys.stderr, flush=True)

    cell = W.fp64_cell(npl=args.npl)
    res = {}
    precs = ["fp64", "mixed", "mixed_stress"] if args.precision == "all" else [args.precision]
    for prec in precs:
        res[prec] = run_plan(sq, [cell], prec, args.steps, args.warmup, use_graph=graph)
        if graph:
            # graph replays record no per-phase events: the kernel times come
            # from an eager run of the same kernels (same stream, HIP events)
            eag = run_plan(sq, [cell], prec, min(args.steps, 3), 1)
            res[prec]["phases"] = eag["phases"]
            res[prec]["eager_ms"] = eag["ms"]
        print("bench: 64000-node cell %s %.2f ms/step  phases %s" % (
            prec, res[prec]["ms"], {k: round(v, 3) for k, v in per_launch(res[prec]).items()}),
            file=sys.stderr, flush=True)

    head = precs[0]
    r = res[head]
    info = r["info"][0]
    Nd = int(info[0])
    fp64 = head == "fp64"
    flops = kernel_flops(info, stress_fp64=fp64)
    pl = per_launch(r)
    dom = max(flops, key=lambda k: pl[k])
    achieved = flops[dom] / (pl[dom] * 1e-3) / 1e12
    wl = "64000-node cell, 21^3 cubes, degree %d" % int(info[2])
    # LDS: FP64 mirror elements are 16 bytes (two planes), FP32 ones 8 bytes
    word = 8 if fp64 or (head == "mixed_stress" and dom != "stress") else 4
    lds_w = 16 if word == 8 else 8
    lds_tbps = lds_bytes(info, word)[dom] / (pl[dom] * 1e-3) / 1e12
    hb_launch, hb_step = hbm_bytes(info)
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
        "dtype": "f64" if fp64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "periodic 16 Bohr cube, h 0.4 (40^3 = 64000 nodes), 64 atoms "
                               "(seed 1, min spacing 1.5), R_cut 4 (21^3 cubes), degree %d, "
                               "kT 0.05 Ha, 12th-order FD, Lanczos K=%d" % (int(info[2]), int(info[9])),
                   "nodes": Nd, "cube": int(info[1]) ** 3, "npl": int(info[2]), "precision": head,
                   "launch": "graph replay" if graph else "eager"},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_F64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_F64_TFLOPS,
                     "traffic": recorded_traffic(dom, head, wl),
                     "algorithmic_flop_per_launch": flops[dom], "launch_ms": pl[dom]},
        "lds": {"kernel": dom, "achieved": lds_tbps, "peak": lds_peak[lds_w][0], "unit": "TB/s",
                "frac": lds_tbps / lds_peak[lds_w][0],
                "peak_kind": "measured, conflict-free %d-byte reads (sq_probe_lds)" % lds_w},
        "hbm": {"achieved": hb_step / (r["ms"] * 1e-3) / 1e9, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": hb_step / (r["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                "kind": "algorithmic (compulsory) bytes per step", "bytes_per_step": hb_step,
                "dominant_kernel_bytes_per_launch": hb_launch[dom],
                "measured": measured_hbm(recorded_traffic(dom, head, wl), pl[dom])},
        "phases_ms": pl,
        "eager_ms_per_step": r.get("eager_ms", r["ms"]),
        "setup_s": r["setup_s"],
        "pressure": {"direct": r["p_direct"][0], "trace": r["p_trace"][0], "unit": "Ha/Bohr^3"},
    }
    for mk in ("mixed", "mixed_stress"):
        if mk not in res or head != "fp64":
            continue
        m = res[mk]
        mf = kernel_flops(m["info"][0], stress_fp64=False)
        mpl = per_launch(m)
        out[mk] = {"value": Nd / (m["ms"] * 1e-3), "ms_per_step": m["ms"], "dtype": "f32+f64",
                   "vectors": ("f64 moments from the Lanczos tridiagonal, f32 stress pass"
                               if lanczos_run(m["info"][0])[1] else
                               "f32 both passes" if mk == "mixed" else "f64 moments, f32 stress pass"),
                   "speedup_vs_fp64": r["ms"] / m["ms"], "phases_ms": mpl,
                   "stress_tflops": mf["stress"] / (mpl["stress"] * 1e-3) / 1e12,
                   "mu_diff_vs_fp64": abs(m["mu"][0] - r["mu"][0]),
                   "sigma_diff_vs_fp64": max(abs(a - b) for a, b in zip(m["sigma"][0], r["sigma"][0])),
                   "p_direct_diff_vs_fp64": abs(m["p_direct"][0] - r["p_direct"][0])}

    if args.extra:
        tune = os.path.join(tempfile.gettempdir(), "sq_bench_tune.json")
        # the batch: one warm-up (it captures the graphs) and one timed step;
        # the 512000-node cell: one eager step (40 s; launch overhead is nil)
        extra = {"batched_32_cells": (W.batched_cells(n_cells=32, seed=3),
                                      dict(use_graph=graph, autotune=True, tune_cache=tune), 1),
                 "large_512000_nodes": ([W.large_cell()], dict(use_graph=False), 0)}
        for name, (cells, kw, warm) in extra.items():
            e = {}
            for prec in ("fp64", "mixed"):
                x = run_plan(sq, cells, prec, 1, warm, **kw)
                e[prec] = {"value": x["nodes"] / (x["ms"] * 1e-3), "ms_per_step": x["ms"],
                           "setup_s": x["setup_s"]}
                print("bench: %s %s %.1f ms/step (set-up %.1f s)" % (name, prec, x["ms"], x["setup_s"]),
                      file=sys.stderr, flush=True)
                if prec == "fp64":
                    s64 = x["sigma"]
                else:
                    e["sigma_diff_vs_fp64"] = max(abs(a - b) for s, t in zip(x["sigma"], s64)
                                                  for a, b in zip(s, t))
                e["nodes"] = x["nodes"]
            e["speedup_mixed_vs_fp64"] = e["fp64"]["ms_per_step"] / e["mixed"]["ms_per_step"]
            e["unit"] = "node-columns/s"
            e["launch"] = ("graph replay" if kw.get("use_graph") else "eager") + \
                (", autotuned" if kw.get("autotune") else "")
            e["steps"] = 1
            e["warmup"] = warm
            out[name] = e

    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(cell, r["mu"][0], args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
