"""CPU checks of the route the GPU takes to the Chebyshev moments when a plan
runs enough Lanczos steps: k Lanczos steps from w give the tridiagonal T
(alpha_1..alpha_k, beta_1..beta_k) of H on the Krylov space of w, and
w^T p(H) w = e_1^T p(T') e_1 for every polynomial of degree <= 2k, with T'
the (k + 1) x (k + 1) extension of T whose last diagonal entry never enters.
So rho^j = w^T T_j(Hhat) w (Sec. IV) follows from a recurrence on T' for
j <= 2k.

* On a random symmetric stencil-like matrix, against the three-term
  recurrence on the matrix itself (plain Lanczos, no reorthogonalisation,
  as the kernels run it); the extension's last entry never enters, and a
  shorter run misses the degrees beyond twice its length.
* On every node of the 12^3 cell and sampled nodes of a 21^3-cube cell,
  against the oracle's moments (recurrence on the cube, Sec. IV) at the
  oracle's own bounds."""

import numpy as np

from oracle import oracle as O
from paper_2006_03697_amd import workloads as W


def _lanczos(H, w, k):
    """Plain Lanczos: alpha_1..alpha_k, beta_1..beta_k (beta_k the norm of the
    last residual)."""
    a, b = np.zeros(k), np.zeros(k)
    q_prev = np.zeros_like(w)
    q = w / np.linalg.norm(w)
    beta = 0.0
    for i in range(k):
        r = H @ q - beta * q_prev
        a[i] = q @ r
        r = r - a[i] * q
        beta = np.linalg.norm(r)
        b[i] = beta
        q_prev, q = q, r / beta
    return a, b


def _quad_moments(a, b, k, chi, zeta, npl, last=0.0):
    """e_1^T T_j(That') e_1, j = 0..npl, from the (k + 1)-dimensional
    extension (its last diagonal entry `last`, scaled)."""
    d = np.concatenate([(a[:k] - chi) / zeta, [last]])
    off = b[:k] / zeta
    T = np.diag(d) + np.diag(off, 1) + np.diag(off, -1)
    t0 = np.zeros(k + 1)
    t0[0] = 1.0
    t1 = T @ t0
    m = [t0[0], t1[0]]
    for _ in range(2, npl + 1):
        t0, t1 = t1, 2.0 * (T @ t1) - t0
        m.append(t1[0])
    return np.array(m)


def _recurrence_moments(H, w, chi, zeta, npl):
    Hh = (H - chi * np.eye(len(w))) / zeta
    t0 = w.copy()
    t1 = Hh @ t0
    m = [w @ t0, w @ t1]
    for _ in range(2, npl + 1):
        t0, t1 = t1, 2.0 * (Hh @ t1) - t0
        m.append(w @ t1)
    return np.array(m)


def test_quadrature_moments_of_a_random_symmetric_matrix():
    rng = np.random.default_rng(11)
    n = 343
    # 7^3 grid Laplacian-like stencil plus a random diagonal and a low-rank term
    L1 = np.diag(np.full(7, 2.0)) - np.diag(np.ones(6), 1) - np.diag(np.ones(6), -1)
    I = np.eye(7)
    H = (np.kron(np.kron(L1, I), I) + np.kron(np.kron(I, L1), I) + np.kron(np.kron(I, I), L1))
    H += np.diag(rng.uniform(-1.0, 1.0, n))
    v = rng.standard_normal((n, 3))
    H += v @ v.T * 0.05
    lam = np.linalg.eigvalsh(H)
    chi, zeta = 0.5 * (lam[-1] + lam[0]), 0.5 * (lam[-1] - lam[0]) * 1.01
    w = np.zeros(n)
    w[171] = 1.0
    k = 20
    a, b = _lanczos(H, w, k)
    ref = _recurrence_moments(H, w, chi, zeta, 2 * k + 1)
    q = _quad_moments(a, b, k, chi, zeta, 2 * k + 1)
    assert np.max(np.abs(q[: 2 * k + 1] - ref[: 2 * k + 1])) < 1e-12
    # the extension's diagonal entry does not enter up to degree 2k (not
    # even in rounding) ...
    q2 = _quad_moments(a, b, k, chi, zeta, 2 * k + 1, last=0.7)
    assert np.max(np.abs(q2[: 2 * k + 1] - q[: 2 * k + 1])) == 0.0
    # ... and a shorter run is exact to twice its length, not beyond (8
    # steps, before the run has converged: degrees 17 and 18 miss by > 1e-3)
    q8 = _quad_moments(a, b, 8, chi, zeta, 18)
    assert np.max(np.abs(q8[:17] - ref[:17])) < 1e-12
    assert abs(q8[17] - ref[17]) > 1e-3 and abs(q8[18] - ref[18]) > 1e-3


def _check_cell(cell, nodes, tol):
    npl = cell["npl"]
    K = max(20, -(-npl // 2))
    ob = O.OracleCell(dict(cell, lanczos_steps=20))
    lo, hi, chi, zeta = ob.bounds(nodes)
    ref = ob.moments(nodes, chi, zeta)
    ol = O.OracleCell(dict(cell, lanczos_steps=K))
    al, be, st = ol.lanczos(nodes)
    # the first 20 steps of the longer run are those of the bounds' run
    a20, b20, s20 = ob.lanczos(nodes)
    assert np.array_equal(al[:, :20], a20) and np.array_equal(be[:, :20], b20)
    worst = 0.0
    for i in range(len(nodes)):
        q = _quad_moments(al[i], be[i], int(st[i]), chi[i], zeta[i], npl)
        worst = max(worst, float(np.max(np.abs(q - ref[i]))))
    assert worst < tol, worst
    return worst


def test_quadrature_moments_match_the_oracle_on_the_12_cube_cell():
    cell = W.tiny_cell(npl=60)   # 30 Lanczos steps on 9^3 cubes
    _check_cell(cell, np.arange(12 ** 3), 1e-12)


def test_quadrature_moments_match_the_oracle_on_21_cubes():
    cell = W.fp64_cell()         # degree 60: 30 Lanczos steps on 21^3 cubes
    _check_cell(cell, W.node_sample(64000, 16, seed=44), 1e-12)
