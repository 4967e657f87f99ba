"""Dense, Kronecker-product constructions of the nodal operators of Sec. IV,
used only to pin the oracle.  They are assembled from 1D matrices and numpy
broadcasting -- a different route from the oracle's point loops."""

import numpy as np


def fd_1d(nc, weights, antisym):
    """Restricted 1D FD matrix on nc points: entries w_|k| on the k-th
    diagonals (antisymmetric: +w_k above, -w_k below); rows lose the entries
    whose column falls outside (the restriction)."""
    A = np.zeros((nc, nc))
    M = len(weights) - 1
    for k in range(0 if not antisym else 1, M + 1):
        if k == 0:
            A += weights[0] * np.eye(nc)
            continue
        up = np.eye(nc, k=k)
        dn = np.eye(nc, k=-k)
        A += weights[k] * up + (-weights[k] if antisym else weights[k]) * dn
    return A


def kron3(A, axis, nc):
    """Lift a 1D operator to the cube; cube index = ix + nc (iy + nc iz)."""
    I = np.eye(nc)
    mats = [I, I, I]
    mats[axis] = A
    # index order x fastest -> kron(z, y, x)
    return np.kron(mats[2], np.kron(mats[1], mats[0]))


def cube_coords(q3, m, h):
    a = np.arange(-m, m + 1)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    # flatten with x fastest
    pts = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                    Z.transpose(2, 1, 0).ravel()], axis=1)
    return (pts + np.asarray(q3)[None, :]) * h


def projectors(coords, images, p_sigma, p_rcut):
    """Columns chi_I (sampled Gaussian, spherical cutoff) for every image that
    reaches a cube node."""
    cols, cen = [], []
    for R in images:
        d = coords - R[None, :]
        d2 = np.einsum("ij,ij->i", d, d)
        chi = np.where(d2 < p_rcut * p_rcut, np.exp(-d2 / (2 * p_sigma ** 2)), 0.0)
        if np.any(chi != 0.0):
            cols.append(chi)
            cen.append(R)
    return np.array(cols).reshape(-1, coords.shape[0]), np.array(cen).reshape(-1, 3)
