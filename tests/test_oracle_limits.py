"""Pins of the FP64 CPU oracle against limits it must reach and published
constants (CPU only):

* jellium (no atoms): the truncated-cube result from 1-D eigendecompositions
  (the nodal Hamiltonian is a Kronecker sum of 1-D Toeplitz matrices), and
  its R_cut -> infinity limit, the Brillouin-zone integral of the kinetic
  stress of the infinite finite-difference crystal (Sec. III/IV: the
  infinite-cell formulation gives the infinite crystal);
* the Perdew-Wang 1992 correlation energy of the uniform gas: its
  high-density (Gell-Mann--Brueckner) and low-density expansion constants.
"""

import math

import numpy as np
import pytest

import _dense as D
from oracle import oracle as O
from paper_2006_03697_amd import workloads as W


def _fermi(x, mu, kT):
    return 0.5 * (1.0 - np.tanh((x - mu) / (2.0 * kT)))


def _jellium(h, rcut, kT, npl, mu, L=4.0):
    """A cell without atoms (uniform zero potential), Fermi level fixed."""
    return W.make_cell(L, h, np.zeros((0, 3)), rcut, npl, kT, mu_mode="fixed", mu=mu, n_electrons=0.0)


def _cube_exact(h, nc, kT, mu, c2, c1):
    """rho_q dV / 2, e_q / 2 and K(q) / 2 of the cube of width nc around a
    node in jellium, with f itself (no Chebyshev truncation): H_q =
    T (+) T (+) T with T the restricted 1-D kinetic matrix, so every
    quantity is a triple sum over the 1-D eigenpairs."""
    m = nc // 2
    T = -0.5 / h ** 2 * D.fd_1d(nc, c2, False)
    G = D.fd_1d(nc, c1, True) / h
    lam, Q = np.linalg.eigh(T)
    e = Q[m, :]                      # <e_c, q_i>
    ge = (G @ Q)[m, :]               # <e_c, G q_i>
    g2e = (G @ G @ Q)[m, :]          # <e_c, G^2 q_i>
    lam3 = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    f = _fermi(lam3, mu, kT)
    w0 = e * e
    rho = np.einsum("ijk,i,j,k->", f, w0, w0, w0)
    en = np.einsum("ijk,i,j,k->", lam3 * f, w0, w0, w0)
    kxx = np.einsum("ijk,i,j,k->", f, g2e * e, w0, w0)
    kxy = np.einsum("ijk,i,j,k->", f, ge * e, ge * e, w0)
    return rho, en, kxx, kxy


def _bz_limit(h, kT, mu, c2, c1, nk):
    """Per node of the infinite grid: D_qq = (h^3 / (2 pi)^3) int_BZ f(eps)
    and (G_x G_x D)_qq = -(h^3 / (2 pi)^3) int_BZ g_x^2 f(eps), with
    eps(k) = sum_a s(k_a) / 2 (s the symbol of minus the 12th-order second
    difference) and i g the symbol of the first difference, by the periodic
    trapezoid rule on nk^3 points (exponentially accurate: the integrand is
    smooth and periodic)."""
    th = 2.0 * np.pi * (np.arange(nk) + 0.5) / nk - np.pi     # k h on a shifted uniform grid
    kk = np.arange(1, len(c2))
    s = -(c2[0] + 2.0 * np.cos(np.outer(th, kk)) @ c2[1:]) / h ** 2
    g = 2.0 * (np.sin(np.outer(th, kk)) @ c1[1:]) / h
    eps = 0.5 * (s[:, None, None] + s[None, :, None] + s[None, None, :])
    f = _fermi(eps, mu, kT)
    w = 1.0 / nk ** 3          # (h^3 / (2 pi)^3) d^3k = d^3(kh) / (2 pi)^3
    rho = np.sum(f) * w
    kxx = -np.sum(f * (g ** 2)[:, None, None]) * w
    return rho, kxx


def test_jellium_cube_matches_kronecker_eigendecomposition():
    h, rcut, kT, mu, npl = 0.5, 3.0, 1.0, 0.3, 320
    cell = _jellium(h, rcut, kT, npl, mu)
    c2, c1 = O.fd_weights(6)
    r = O.run(cell, nodes=[0], mu=mu)
    nc = 2 * int(math.floor(rcut / h + 1e-9)) + 1
    rho, en, kxx, kxy = _cube_exact(h, nc, kT, mu, c2, c1)
    rec = r["records"][0]
    dV = h ** 3
    assert abs(rec[0] * dV / 2 - rho) < 1e-11 * rho
    assert abs(rec[1] / 2 - en) < 1e-10 * abs(en)
    K = rec[2:11].reshape(3, 3) / 2
    scale = abs(kxx)
    for a in range(3):
        assert abs(K[a, a] - kxx) < 1e-10 * scale
        for b in range(3):
            if a != b:
                assert abs(K[a, b] - kxy) < 1e-10 * scale
    # the uniform cube has cubic symmetry: the off-diagonal part vanishes
    assert abs(kxy) < 1e-13 * scale
    # no atoms, no nonlocal stress
    assert np.all(rec[11:21] == 0.0)


def test_jellium_kinetic_stress_reaches_the_brillouin_zone_limit():
    h, kT, mu = 0.5, 1.0, 0.3
    c2, c1 = O.fd_weights(6)
    rho_bz, kxx_bz = _bz_limit(h, kT, mu, c2, c1, 64)
    rho_bz2, kxx_bz2 = _bz_limit(h, kT, mu, c2, c1, 96)
    # the quadrature has converged
    assert abs(rho_bz - rho_bz2) < 1e-14 and abs(kxx_bz - kxx_bz2) < 1e-12 * abs(kxx_bz)
    # the truncated cube converges to it exponentially in R_cut
    errs = []
    for nc in (9, 13, 17, 25, 33):
        rho, en, kxx, kxy = _cube_exact(h, nc, kT, mu, c2, c1)
        errs.append(abs(kxx - kxx_bz) / abs(kxx_bz))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-10, errs
    # the oracle itself (Chebyshev quadrature on its 25^3 cube) at the limit
    cell = _jellium(h, 6.0, kT, 400, mu)
    r = O.run(cell, nodes=[0], mu=mu)
    rec = r["records"][0]
    assert abs(rec[0] * h ** 3 / 2 - rho_bz) < 1e-8 * rho_bz
    assert abs(rec[2] / 2 - kxx_bz) < 1e-8 * abs(kxx_bz)
    # sigma^I_aa / |Omega| of the oracle's cell = N_d K(q) / |Omega| = K(q) / h^3 < 0
    assert rec[2] < 0


# ----------------------------------------------------------------------------
# Perdew-Wang 1992 correlation (unpolarised): the fit is built to reproduce
# the uniform-gas expansions
#   high density  eps_c = c0 ln rs - c1 + c2 rs ln rs + O(rs),
#                 c0 = (1 - ln 2)/pi^2 (A = 0.031091 in the fit),
#                 c1 = 0.046644, c2 = 0.00664
#                 (no sqrt(rs) term: that fixes b2 = 2 c0 b1^2, and c1 fixes
#                 b1 = exp(-c1 / (2 c0)) / (2 c0));
#   low density   eps_c = -d0 / rs + d1 / rs^(3/2) + ..., d0 = 0.4335,
#                 d1 = 1.4408
# (Perdew & Wang, Phys. Rev. B 45, 13244 (1992), the constants of their
# Table I for the unpolarised gas).  a1, b3 and b4 are fitted to Monte-Carlo
# data; the expansions fix the combinations a1/b4 and a1 b3/b4^2, the value
# of a1 itself only through c2 (three printed digits).
# ----------------------------------------------------------------------------

def _eps_c(rs):
    rho = 3.0 / (4.0 * np.pi * rs ** 3)
    return O.lda_parts(rho)[2]


def test_pw92_high_density_expansion():
    # the fit's A is c0 rounded to five figures
    c0 = (1.0 - math.log(2.0)) / math.pi ** 2
    A = 0.031091
    assert abs(A - c0) < 5e-7
    # -c1: the constant term, from tiny rs (the rs ln rs term is below 1e-9);
    # 0.046644 is printed to six decimals and b1 to five figures
    for rs in (1e-8, 1e-7):
        assert abs(_eps_c(rs) - A * math.log(rs) + 0.046644) < 2e-6
    # the coefficient of ln rs is A: the constant term does not drift
    # over six decades of rs
    k = [_eps_c(rs) - A * math.log(rs) for rs in (1e-12, 1e-9, 1e-6)]
    assert abs(k[0] - k[1]) < 1e-8 and abs(k[1] - k[2]) < 2e-6
    c1 = -k[0]
    # (eps - A ln rs + c1) / rs = a rs^-1/2 + c2 ln rs - c3 + O(rs^1/2): a
    # least-squares fit over five decades separates the terms.  c2 is the
    # rs ln rs coefficient; a is what a b2 off the constraint
    # b2 = 2 A b1^2 leaves (only the rounding of the printed b1, b2 here)
    rs = np.logspace(-8, -3, 16)
    f = np.array([(_eps_c(r) - A * math.log(r) + c1) / r for r in rs])
    B = np.stack([rs ** -0.5, np.log(rs), np.ones_like(rs), rs ** 0.5, rs * np.log(rs), rs], 1)
    a, c2 = np.linalg.lstsq(B, f, rcond=None)[0][:2]
    assert abs(c2 - 0.00664) < 1e-5, c2
    assert abs(a) < 1e-6, a


def test_pw92_low_density_expansion():
    # eps = -d0 / rs + d1 / rs^(3/2) + O(rs^-2): a least-squares fit over
    # rs in [1e3, 1e5] (above that ln(1 + 1/Q) in double precision loses the
    # digits the fit needs)
    rs = np.logspace(3, 5, 16)
    B = np.stack([-1.0 / rs, rs ** -1.5, rs ** -2.0, rs ** -2.5, rs ** -3.0], 1)
    d0, d1 = np.linalg.lstsq(B, [_eps_c(r) for r in rs], rcond=None)[0][:2]
    assert abs(d0 - 0.4335) < 1e-4, d0
    assert abs(d1 - 1.4408) < 1e-3, d1
