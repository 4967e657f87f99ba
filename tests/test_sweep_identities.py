"""CPU checks of the algebra the GPU kernels rely on (no GPU, no oracle):

* one projector sweep per operator application: every column visits its
  images in increasing index and takes the projection onto chi_I before it
  adds c_I chi_I; summed over the columns this gives
  <chi_I, u> + sum_{J < I} c_J G_IJ, and the upper triangle of the Gram
  matrix G_IJ = <chi_I, chi_J> restores <chi_I, u + sum_J c_J chi_J>;
* Clenshaw's recurrence for d = sum'_j c_j T_j(A) w equals the forward
  three-term recurrence with the sum accumulated."""

import numpy as np


def _random_projectors(rng, ncol, nz, nimg):
    """Columns x planes x images: each image covers a random contiguous chord
    on a random subset of columns (the shape of spherical supports)."""
    chi = np.zeros((ncol, nz, nimg))
    for i in range(nimg):
        cols = rng.choice(ncol, size=rng.integers(1, ncol), replace=False)
        for c in cols:
            z0 = rng.integers(0, nz)
            z1 = rng.integers(z0, nz)
            chi[c, z0:z1 + 1, i] = rng.uniform(0.1, 1.0, z1 - z0 + 1)
    return chi


def test_single_sweep_projections_with_the_gram_upper_triangle():
    rng = np.random.default_rng(5)
    ncol, nz, nimg = 40, 21, 12
    chi = _random_projectors(rng, ncol, nz, nimg)
    u = rng.standard_normal((ncol, nz))
    c = rng.standard_normal(nimg)
    # the sweep as each column performs it
    io = u.copy()
    proj = np.zeros(nimg)
    for col in range(ncol):
        for i in range(nimg):                       # increasing image index
            w = chi[col, :, i]
            if not w.any():
                continue
            proj[i] += w @ io[col]                  # projection first
            io[col] += c[i] * w                     # then the projector term
    G = np.einsum("czi,czj->ij", chi, chi)
    corr = np.array([sum(G[i, j] * c[j] for j in range(i, nimg)) for i in range(nimg)])
    exact_vec = u + np.einsum("czi,i->cz", chi, c)
    exact = np.einsum("czi,cz->i", chi, exact_vec)
    assert np.allclose(io, exact_vec, rtol=0, atol=1e-12)
    assert np.max(np.abs(proj + corr - exact)) < 1e-12 * np.max(np.abs(exact))
    # without the correction the sweep is wrong: the check is not vacuous
    assert np.max(np.abs(proj - exact)) > 1e-3 * np.max(np.abs(exact))


def test_clenshaw_equals_the_forward_recurrence():
    rng = np.random.default_rng(7)
    n, npl = 30, 17
    M = rng.standard_normal((n, n))
    A = (M + M.T) / (2 * np.linalg.norm(M, 2))       # spectrum inside [-1, 1]
    w = np.zeros(n)
    w[n // 2] = 1.0
    c = rng.standard_normal(npl + 1)
    # forward: t^{j+1} = 2 A t^j - t^{j-1}, d = sum' c_j t^j
    t0, t1 = w.copy(), A @ w
    d = 0.5 * c[0] * t0 + c[1] * t1
    for j in range(2, npl + 1):
        t0, t1 = t1, 2 * A @ t1 - t0
        d += c[j] * t1
    # Clenshaw: b_k = c_k w + 2 A b_{k+1} - b_{k+2}, d = c_0 w / 2 + A b_1 - b_2
    b1, b2 = c[npl] * w, np.zeros(n)
    for k in range(npl - 1, 0, -1):
        b1, b2 = c[k] * w + 2 * A @ b1 - b2, b1
    dc = 0.5 * c[0] * w + A @ b1 - b2
    assert np.max(np.abs(dc - d)) < 1e-12 * np.max(np.abs(d))
