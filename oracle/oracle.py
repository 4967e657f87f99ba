"""FP64 CPU oracle for the infinite-cell Clenshaw-Curtis SQ hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the HIP path (``paper_2006_03697_amd``): grid, images, local
potential, FD weights, spectral bounds, quadrature coefficients, Fermi level,
density, band energy and stress are all recomputed here, with plain loops in
``sq_oracle.c`` and plain numpy / scipy steps below.

Paper: Sharma, Hamel, Bethkenhagen, Pask, Suryanarayana, arXiv 2006.03697.
  * density matrix, rho = 2 D(x, x)                         -- Sec. III
  * kinetic / nonlocal DM stress sigma^I, sigma^III          -- Sec. III
  * nodal Hamiltonian H_q on the cube of side 2 R_cut        -- Sec. IV
  * Hhat_q = (H_q - chi_q)/zeta_q, chi/zeta from the extreme
    eigenvalues of H_q                                       -- Sec. IV
  * Clenshaw-Curtis coefficients c_q^j of the Fermi-Dirac
    function, primed sum, three-term recurrence t_q^j        -- Sec. IV
  * rho_q = (2/dV) sum' c_q^j rho_q^j, rho_q^j = w_q^T t_q^j   -- Sec. IV
  * band-energy trace sum'(chi_q c_q^j + zeta_q d_q^j) rho_q^j -- App. A
  * SQ kinetic + nonlocal stress                             -- Sec. IV
  * direct pressure from the band energy, no second
    derivatives of the density matrix                        -- App. A

Readings of what the paper leaves open (also listed in the design notes):
  R1 spectral bounds: K-step FP64 Lanczos from w_q, no reorthogonalisation,
     extreme Ritz values widened by their residuals beta_K |s_K,i|;
  R2 c_q^j by the M_q-point Gauss-Chebyshev rule, M_q the smallest power of
     two >= max(4 (n_pl + 2), 8 zeta_q / kT);
  R3 mu solves 2 sum_q sum' c_q^j(mu) rho_q^j = N_e (bisection on the
     spectral bracket widened by 40 kT on each side), or is fixed;
  R5 d_q^j are the Chebyshev coefficients of r g(r);
  R8 spherical cutoffs of the Gaussian potential / projector;
  R16 the direct pressure keeps only the kinetic and nonlocal terms: the
     kinetic trace from the band energy with the local and nonlocal
     potential energies taken back out, plus tr N;
  R17 LDA exchange-correlation: Slater exchange, Perdew-Wang 1992
     correlation (unpolarised); nodes with rho <= 0 contribute nothing.
Parity unpinned (problem-definition choices, no external value fixes them):
the Lanczos step count / widening rule (R1) and the cutoffs (R8).  The
Perdew-Wang parameters are pinned through the uniform-gas expansion
constants they were fitted to reproduce (A, b1, b2 by the high-density
c0, c1 and the absent sqrt(rs) term; a1, b3, b4 by c2, d0 = a1/b4 and
d1 = a1 b3/b4^2, to the digits those constants are printed with).
"""

from __future__ import annotations

import ctypes
import math
import os
from fractions import Fraction

import numpy as np
from scipy.linalg import eigh_tridiagonal

from . import build as _build

SP_KEYS = ("v_amp", "v_sigma", "v_rcut", "p_sigma", "p_rcut", "gamma", "z_val")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


class _CCell(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double), ("L", ctypes.c_double * 3),
                ("m", ctypes.c_int), ("M", ctypes.c_int), ("c2", _dp), ("c1", _dp),
                ("vloc", _dp), ("nimg", ctypes.c_int), ("img", _dp), ("img_sp", _ip),
                ("sp", _dp)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        cp = ctypes.POINTER(_CCell)
        L.or_node_lanczos.argtypes = [cp, ctypes.c_long, ctypes.c_int, _dp, _dp, _dp]
        L.or_node_lanczos.restype = ctypes.c_int
        L.or_node_moments.argtypes = [cp, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, _dp]
        L.or_node_stress.argtypes = [cp, ctypes.c_long, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, _dp, _dp, _dp]
        L.or_node_dense_H.argtypes = [cp, ctypes.c_long, _dp]
        L.or_node_counts.argtypes = [cp, ctypes.c_long, _ip, _ip]
        L.or_vloc.argtypes = [cp, _dp]
        L.or_node_projector_sums.argtypes = [cp, ctypes.c_long, ctypes.c_int, _ip, _dp]
        L.or_node_projector_sums.restype = ctypes.c_int
        L.or_batch_lanczos.argtypes = [cp, _lp, ctypes.c_long, ctypes.c_int, _dp, _dp, _ip]
        L.or_batch_moments.argtypes = [cp, _lp, ctypes.c_long, _dp, _dp, ctypes.c_int, _dp]
        L.or_batch_stress.argtypes = [cp, _lp, ctypes.c_long, _dp, _dp, ctypes.c_int, _dp, _dp]
        _LIB = L
    return _LIB


def _p(a, t=_dp):
    return a.ctypes.data_as(t)


# ---------------------------------------------------------------------------
# finite differences
# ---------------------------------------------------------------------------

def fd_weights(M: int):
    """Central finite-difference weights of order 2M (the paper uses 12th
    order, M = 6; Sec. V).  Closed form in exact rationals:
        second derivative  c_k = 2 (-1)^(k+1) (M!)^2 / (k^2 (M-k)! (M+k)!),
                           c_0 = -2 sum_{k>=1} c_k
        first derivative   w_k = (-1)^(k+1) (M!)^2 / (k (M-k)! (M+k)!)
    Returns (c2[0..M], c1[0..M]) as float64 (c1[0] = 0)."""
    f = math.factorial
    c2 = [Fraction(0)] * (M + 1)
    c1 = [Fraction(0)] * (M + 1)
    for k in range(1, M + 1):
        base = Fraction(f(M) ** 2, f(M - k) * f(M + k))
        sgn = 1 if k % 2 == 1 else -1
        c2[k] = 2 * sgn * base / (k * k)
        c1[k] = sgn * base / k
    c2[0] = -2 * sum(c2[1:])
    return (np.array([float(x) for x in c2]), np.array([float(x) for x in c1]))


# ---------------------------------------------------------------------------
# cell geometry
# ---------------------------------------------------------------------------

class OracleCell:
    """One periodic orthorhombic cell prepared for the per-node SQ oracle."""

    def __init__(self, cell: dict):
        self.cell = cell
        L = np.array(cell["L"], dtype=np.float64)
        h = float(cell["h"])
        nf = L / h
        n = np.rint(nf).astype(int)
        if np.any(np.abs(nf - n) > 1e-9 * nf):
            raise ValueError("cell side is not an integer number of mesh steps")
        self.L, self.h, self.n = L, h, n
        self.Nd = int(np.prod(n))
        self.dV = h ** 3
        self.volume = float(np.prod(L))
        self.m = int(math.floor(cell["rcut"] / h + 1e-9))
        if self.m < 1:
            raise ValueError("R_cut must be at least one mesh step")
        self.nc = 2 * self.m + 1
        self.M = int(cell["fd_half_order"])
        self.c2, self.c1 = fd_weights(self.M)
        self.npl = int(cell["npl"])
        self.kT = float(cell["kT"])
        self.K = int(cell.get("lanczos_steps", 20))
        sp = np.array([[s[k] for k in SP_KEYS] for s in cell["species_params"]], dtype=np.float64)
        self.sp = np.ascontiguousarray(sp)
        pos = np.asarray(cell["pos"], dtype=np.float64).reshape(-1, 3)
        pos = pos - L * np.floor(pos / L)          # wrap into [0, L)
        self.pos = pos
        self.species = np.asarray(cell["species"], dtype=np.int32)
        self._images()
        self._make_struct(vloc=np.zeros(1))
        self.vloc = np.zeros(self.Nd)
        lib().or_vloc(ctypes.byref(self.cs), _p(self.vloc))
        self._make_struct(vloc=self.vloc)

    def _images(self):
        """All periodic images R_I + n L within the species' reach of the box
        spanned by every node's cube (infinite-cell formulation, Sec. IV)."""
        h, m, n, L = self.h, self.m, self.n, self.L
        reach = float(max(max(s[2], s[4]) for s in self.sp))
        lo = -m * h - reach
        hi = (n - 1 + m) * h + reach
        imgs, sps = [], []
        for I in range(self.pos.shape[0]):
            p = self.pos[I]
            rng = [range(int(math.floor((lo - p[a]) / L[a])) - 1,
                         int(math.ceil((hi[a] - p[a]) / L[a])) + 2) for a in range(3)]
            for i in rng[0]:
                for j in rng[1]:
                    for k in rng[2]:
                        R = p + np.array([i, j, k], dtype=np.float64) * L
                        box_lo = -m * h
                        box_hi = (n - 1 + m) * h
                        e = np.maximum(box_lo - R, 0.0) + np.maximum(R - box_hi, 0.0)
                        if float(np.dot(e, e)) < reach * reach:
                            imgs.append(R)
                            sps.append(self.species[I])
        self.img = np.ascontiguousarray(np.array(imgs, dtype=np.float64).reshape(-1, 3))
        self.img_sp = np.ascontiguousarray(np.array(sps, dtype=np.int32))

    def _make_struct(self, vloc):
        self._keep = [self.c2, self.c1, vloc, self.img, self.img_sp, self.sp]
        cs = _CCell()
        cs.n = (ctypes.c_int * 3)(*[int(x) for x in self.n])
        cs.h = self.h
        cs.L = (ctypes.c_double * 3)(*[float(x) for x in self.L])
        cs.m = self.m
        cs.M = self.M
        cs.c2 = _p(self.c2)
        cs.c1 = _p(self.c1)
        cs.vloc = _p(vloc)
        cs.nimg = int(self.img.shape[0])
        cs.img = _p(self.img)
        cs.img_sp = _p(self.img_sp, _ip)
        cs.sp = _p(self.sp)
        self.cs = cs

    # -- per-node building blocks ---------------------------------------------

    def nodes_all(self) -> np.ndarray:
        return np.arange(self.Nd, dtype=np.int64)

    def dense_H(self, q: int) -> np.ndarray:
        Nc = self.nc ** 3
        H = np.zeros((Nc, Nc))
        lib().or_node_dense_H(ctypes.byref(self.cs), int(q), _p(H))
        return H

    def counts(self, q: int):
        a = ctypes.c_int()
        b = ctypes.c_int()
        lib().or_node_counts(ctypes.byref(self.cs), int(q), ctypes.byref(a), ctypes.byref(b))
        return a.value, b.value

    def projector_sums(self, q: int):
        cap = 4096
        img = np.zeros(cap, dtype=np.int32)
        sums = np.zeros(cap)
        k = lib().or_node_projector_sums(ctypes.byref(self.cs), int(q), cap, _p(img, _ip), _p(sums))
        return img[:k].copy(), sums[:k].copy()

    def lanczos(self, nodes):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        n = nodes.shape[0]
        al = np.zeros((n, self.K))
        be = np.zeros((n, self.K))
        st = np.zeros(n, dtype=np.int32)
        lib().or_batch_lanczos(ctypes.byref(self.cs), _p(nodes, _lp), n, self.K, _p(al), _p(be),
                               _p(st, _ip))
        return al, be, st

    def bounds(self, nodes):
        """(lam_lo, lam_hi, chi, zeta) per node (reading R1)."""
        al, be, st = self.lanczos(nodes)
        lo = np.zeros(len(st))
        hi = np.zeros(len(st))
        for i, k in enumerate(st):
            lo[i], hi[i] = ritz_bounds(al[i, :k], be[i, :k])
        return lo, hi, 0.5 * (hi + lo), 0.5 * (hi - lo)

    def moments(self, nodes, chi, zeta):
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        zeta = np.ascontiguousarray(zeta, dtype=np.float64)
        mom = np.zeros((nodes.shape[0], self.npl + 1))
        lib().or_batch_moments(ctypes.byref(self.cs), _p(nodes, _lp), nodes.shape[0], _p(chi),
                               _p(zeta), self.npl, _p(mom))
        return mom

    def stress_records(self, nodes, chi, zeta, coef):
        """Per node: K (9), N (9), E_nl density, d_qq."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int64)
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        zeta = np.ascontiguousarray(zeta, dtype=np.float64)
        coef = np.ascontiguousarray(coef[:, : self.npl + 1], dtype=np.float64)
        out = np.zeros((nodes.shape[0], 20))
        lib().or_batch_stress(ctypes.byref(self.cs), _p(nodes, _lp), nodes.shape[0], _p(chi),
                              _p(zeta), self.npl, _p(coef), _p(out))
        return out

    def dm_column(self, q, chi, zeta, coef):
        """Full DM column d_q on the cube (for tests on tiny cubes)."""
        Nc = self.nc ** 3
        d = np.zeros(Nc)
        out = np.zeros(20)
        c = np.ascontiguousarray(coef[: self.npl + 1], dtype=np.float64)
        lib().or_node_stress(ctypes.byref(self.cs), int(q), float(chi), float(zeta), self.npl,
                             _p(c), _p(out), _p(d))
        return d, out


# ---------------------------------------------------------------------------
# spectral bounds (R1) and quadrature coefficients (Sec. IV, R2, R5)
# ---------------------------------------------------------------------------

def ritz_bounds(alpha, beta):
    """Extreme Ritz values of the Lanczos tridiagonal widened by their
    residual norms beta_K |s_K,i| (s_i the Ritz vectors)."""
    k = len(alpha)
    if k == 1:
        theta = np.array([alpha[0]])
        last = np.array([1.0])
    else:
        theta, S = eigh_tridiagonal(np.asarray(alpha), np.asarray(beta[: k - 1]))
        last = S[-1, :]
    r = beta[k - 1] * np.abs(last)
    return theta[0] - r[0], theta[-1] + r[-1]


def quad_points(zeta: float, kT: float, npl: int) -> int:
    """M_q of reading R2: smallest power of two >= max(4 (npl + 2), 8 zeta / kT)."""
    target = max(4 * (npl + 2), int(math.ceil(8.0 * zeta / kT)))
    M = 1
    while M < target:
        M *= 2
    return M


def fermi(x, mu_hat, sig_hat):
    """Fermi-Dirac occupation g(x) = 1 / (1 + exp((x - mu)/sigma)) in the
    overflow-free form (1 - tanh((x - mu) / (2 sigma))) / 2."""
    return 0.5 * (1.0 - np.tanh((x - mu_hat) / (2.0 * sig_hat)))


def cheb_coeffs(mu_hat, sig_hat, M, jmax):
    """c_j = (2/pi) int g(r) T_j(r) / sqrt(1 - r^2) dr (Sec. IV) and d_j, the
    same for r g(r) (App. A), j = 0..jmax, by the M-point Gauss-Chebyshev rule:
    c_j = (2/M) sum_k g(cos th_k) cos(j th_k), th_k = pi (k + 1/2) / M."""
    th = np.pi * (np.arange(M) + 0.5) / M
    x = np.cos(th)
    g = fermi(x, mu_hat, sig_hat)
    C = np.cos(np.outer(np.arange(jmax + 1), th))
    return (2.0 / M) * (C @ g), (2.0 / M) * (C @ (x * g))


def primed(c, r):
    """sum'_{j} c_j r_j: the first term halved."""
    return 0.5 * c[0] * r[0] + float(np.dot(c[1:], r[1:]))


# ---------------------------------------------------------------------------
# whole-cell driver
# ---------------------------------------------------------------------------

class Result(dict):
    pass


_COS_CACHE = {}


def _cos_table(M, jmax):
    key = (M, jmax)
    if key not in _COS_CACHE:
        th = np.pi * (np.arange(M) + 0.5) / M
        _COS_CACHE[key] = (np.cos(th), np.cos(np.outer(np.arange(jmax + 1), th)))
    return _COS_CACHE[key]


def node_coefficients(oc: OracleCell, mu, chi, zeta):
    """c_q^j and d_q^j for every node at Fermi level mu: the rule of
    ``cheb_coeffs`` applied to all nodes that share the same M_q at once."""
    chi = np.asarray(chi)
    zeta = np.asarray(zeta)
    n = len(chi)
    c = np.zeros((n, oc.npl + 1))
    d = np.zeros((n, oc.npl + 1))
    Ms = np.array([quad_points(z, oc.kT, oc.npl) for z in zeta])
    for M in np.unique(Ms):
        sel = np.nonzero(Ms == M)[0]
        x, C = _cos_table(int(M), oc.npl)
        for a in range(0, len(sel), 4096):
            s = sel[a:a + 4096]
            mu_hat = ((mu - chi[s]) / zeta[s])[:, None]
            sig_hat = (oc.kT / zeta[s])[:, None]
            g = fermi(x[None, :], mu_hat, sig_hat)
            c[s] = (2.0 / M) * (g @ C.T)
            d[s] = (2.0 / M) * ((g * x[None, :]) @ C.T)
    return c, d


def electron_count(oc: OracleCell, mu, chi, zeta, mom) -> float:
    """N(mu) = 2 sum_q sum'_j c_q^j(mu) rho_q^j (reading R3)."""
    c, _ = node_coefficients(oc, mu, chi, zeta)
    return 2.0 * math.fsum(primed(c[i], mom[i]) for i in range(len(chi)))


def solve_mu(oc: OracleCell, lo_b, hi_b, chi, zeta, mom, n_electrons, tol=1e-13, max_it=200):
    """Bisection on [min lambda_lo - 40 kT, max lambda_hi + 40 kT] (the
    smearing tails reach past the spectrum: a dilute cell has its Fermi level
    below every node's lowest eigenvalue); stops when |N - N_e| <= tol N_e
    (the last midpoint is returned) or after max_it halvings (the midpoint of
    the final bracket is returned)."""
    lo = float(np.min(lo_b)) - 40.0 * oc.kT
    hi = float(np.max(hi_b)) + 40.0 * oc.kT
    if not electron_count(oc, lo, chi, zeta, mom) < n_electrons < electron_count(oc, hi, chi, zeta, mom):
        raise RuntimeError("Fermi level not bracketed")
    for it in range(max_it):
        mu = 0.5 * (lo + hi)
        N = electron_count(oc, mu, chi, zeta, mom)
        if abs(N - n_electrons) <= tol * n_electrons:
            return mu, it + 1
        if N < n_electrons:
            lo = mu
        else:
            hi = mu
    return 0.5 * (lo + hi), max_it


# ---------------------------------------------------------------------------
# LDA exchange-correlation stress (Sec. II, the exchange-correlation term of
# the stress; for a local functional it is isotropic), reading R17: Slater
# exchange and the Perdew-Wang 1992 parameterisation of the correlation
# energy of the unpolarised uniform electron gas
# ---------------------------------------------------------------------------

def lda_exc(rho):
    """(eps_xc, v_xc): energy per electron and potential for density rho > 0 (Ha)."""
    ex, vx, ec, vc = lda_parts(rho)
    return ex + ec, vx + vc


def lda_parts(rho):
    """(eps_x, v_x, eps_c, v_c) for density rho > 0 (Ha).
    eps_x = -(3/4) (3 rho / pi)^(1/3); v_x = (4/3) eps_x;
    eps_c = -2 A (1 + a1 rs) ln(1 + 1 / (2 A (b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2))),
    rs = (3 / (4 pi rho))^(1/3); v_c = eps_c - (rs / 3) d eps_c / d rs."""
    rho = np.asarray(rho, dtype=np.float64)
    ex = -0.75 * np.cbrt(3.0 * rho / np.pi)
    vx = 4.0 / 3.0 * ex
    A, a1, b1, b2, b3, b4 = 0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294
    rs = np.cbrt(3.0 / (4.0 * np.pi * rho))
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    Q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    ec = Q0 * np.log(1.0 + 1.0 / Q1)
    dec = -2.0 * A * a1 * np.log(1.0 + 1.0 / Q1) - Q0 * Q1p / (Q1 * Q1 + Q1)
    vc = ec - rs / 3.0 * dec
    return ex, vx, ec, vc


def _in_chunks(fn, nodes, per_node, progress, what, chunk=4096):
    """fn(nodes, *per_node) over consecutive chunks of the nodes, results
    stacked (the nodes are independent; chunking only lets a long run report
    its progress)."""
    if progress is None or len(nodes) <= chunk:
        return fn(nodes, *per_node)
    outs = []
    for a in range(0, len(nodes), chunk):
        b = min(a + chunk, len(nodes))
        outs.append(fn(nodes[a:b], *[x[a:b] for x in per_node]))
        progress("%s %d/%d" % (what, b, len(nodes)))
    if isinstance(outs[0], tuple):
        return tuple(np.concatenate([o[k] for o in outs]) for k in range(len(outs[0])))
    return np.concatenate(outs)


def run(cell: dict, nodes=None, mu=None, with_stress=True, progress=None) -> Result:
    """Full SQ evaluation of one cell.

    nodes=None: every node; mu from the electron count unless the cell's
    mu_mode is "fixed" or ``mu`` is given.  With a node subset the Fermi level
    must be given (a subset cannot fix it).

    records[i] = rho_q, band-energy density e_q, K (9), N (9), nonlocal
    energy density, local-potential energy density dV V_q rho_q, LDA
    exchange-correlation energy dV rho_q eps_xc and stress density
    dV rho_q (eps_xc - v_xc).  With the
    stress: sigma = (sum K + sum N) / |Omega| and the pressures
      P_direct = -(-2 E_band + 2 sum_q dV V_q rho_q + 2 E_nl + tr N) / (3 |Omega|)
      P_trace  = -tr(K + N) / (3 |Omega|).

    progress: optional callable given a short message after each chunk of
    nodes of the long stages."""
    oc = OracleCell(cell)
    all_nodes = nodes is None
    nodes = oc.nodes_all() if all_nodes else np.ascontiguousarray(nodes, dtype=np.int64)
    lo, hi, chi, zeta = _in_chunks(oc.bounds, nodes, [], progress, "bounds")
    mom = _in_chunks(oc.moments, nodes, [chi, zeta], progress, "moments")
    it = 0
    if mu is None:
        if cell.get("mu_mode", "solve") == "fixed":
            mu = float(cell["mu"])
        elif all_nodes:
            mu, it = solve_mu(oc, lo, hi, chi, zeta, mom, float(cell["n_electrons"]))
        else:
            raise ValueError("a node subset needs a given Fermi level")
    c, d = node_coefficients(oc, mu, chi, zeta)
    n = len(nodes)
    rec = np.zeros((n, 24))
    for i in range(n):
        rec[i, 0] = 2.0 / oc.dV * primed(c[i], mom[i])
        rec[i, 1] = 2.0 * primed(chi[i] * c[i] + zeta[i] * d[i], mom[i])
        rec[i, 21] = oc.dV * oc.vloc[nodes[i]] * rec[i, 0]
    res = Result(mu=mu, mu_iterations=it, nodes=nodes, lam_lo=lo, lam_hi=hi, chi=chi, zeta=zeta,
                 moments=mom, coef=c, dcoef=d, rho=rec[:, 0].copy(), e_node=rec[:, 1].copy(),
                 volume=oc.volume, dV=oc.dV)
    res["e_band"] = math.fsum(rec[:, 1])
    res["n_count"] = math.fsum(rec[:, 0]) * oc.dV
    # exchange-correlation energy and the isotropic LDA stress term
    # sigma^II = delta_ab sum_q dV rho_q (eps_xc - v_xc) / |Omega| (R17)
    pos = rec[:, 0] > 0.0
    exc = np.zeros(n)
    vxc = np.zeros(n)
    exc[pos], vxc[pos] = lda_exc(rec[pos, 0])
    xc_e = oc.dV * rec[:, 0] * exc
    xc_s = oc.dV * rec[:, 0] * (exc - vxc)
    res["e_xc"] = math.fsum(xc_e)
    res["sigma_xc"] = math.fsum(xc_s) / oc.volume
    rec[:, 22] = xc_e
    rec[:, 23] = xc_s
    if with_stress:
        st = _in_chunks(oc.stress_records, nodes, [chi, zeta, c], progress, "stress")
        rec[:, 2:20] = st[:, 0:18]
        res["e_nl_node"] = st[:, 18].copy()
        parts = np.array([math.fsum(rec[:, 2 + k]) for k in range(18)])
        res["parts"] = parts                    # K (3x3), N (3x3), sums over nodes
        sig = (parts[:9] + parts[9:]).reshape(3, 3) / oc.volume
        res["sigma_full"] = sig
        res["sigma_voigt"] = np.array([sig[0, 0], sig[1, 1], sig[2, 2],
                                       0.5 * (sig[1, 2] + sig[2, 1]),
                                       0.5 * (sig[0, 2] + sig[2, 0]),
                                       0.5 * (sig[0, 1] + sig[1, 0])])
        res["e_nl"] = math.fsum(st[:, 18])
        rec[:, 20] = st[:, 18]
        # direct pressure (App. A) restricted to the kinetic + nonlocal terms:
        # the kinetic trace comes from the band energy with the local and
        # nonlocal potential energies taken back out, the nonlocal part is
        # tr N; the trace form is -tr(K + N) / 3 of the stress
        res["v_rho"] = math.fsum(rec[:, 21])
        trK = parts[0] + parts[4] + parts[8]
        trN = parts[9] + parts[13] + parts[17]
        res["pressure_direct"] = -(-2.0 * res["e_band"] + 2.0 * res["v_rho"] + 2.0 * res["e_nl"]
                                   + trN) / (3.0 * oc.volume)
        res["pressure_trace"] = -(trK + trN) / (3.0 * oc.volume)
    res["records"] = rec
    return res
