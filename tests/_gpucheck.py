"""Comparison and reporting helpers shared by the GPU parity tests."""

import os
import sys

import numpy as np


def report(*a):
    """A line of the parity report: to stderr, and appended to
    $SQ_REPORT_DIR/parity_report.txt when that variable names a folder."""
    print(*a, file=sys.stderr, flush=True)
    d = os.environ.get("SQ_REPORT_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "parity_report.txt"), "a") as f:
            print(*a, file=f)


def moments_excess(mom, lo, hi, ref):
    """Largest difference of the Chebyshev moments rho_q^j of the HIP path
    and of the oracle beyond what the two sides' spectral bounds explain.
    Each side scales H_q by its own (chi_q, zeta_q) from its own Lanczos run;
    these agree to ~1e-12 relative, and since |T_j'(x)| <= j^2 on [-1, 1], a
    shift d_chi, d_zeta moves rho_q^j by at most
    j^2 (|d_chi| + |d_zeta|) / zeta to first order.  The density, energy and
    stress do not depend on the scaling (only through the truncation of a
    converged expansion), the moments at high degree do."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    chi, zeta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    dx = (np.abs(chi - ref["chi"]) + np.abs(zeta - ref["zeta"])) / ref["zeta"]
    j = np.arange(mom.shape[1], dtype=np.float64)
    allow = dx[:, None] * (j * j)[None, :]
    return float(np.max(np.abs(mom - ref["moments"]) - allow))
