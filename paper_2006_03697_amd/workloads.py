"""Seeded synthetic cells for the SQ hot path.

This module only draws atom positions and collects the scalar parameters of a
cell into a plain dict.  It contains none of the method's arithmetic, so both
the CPU oracle (via the tests) and the HIP path can consume what it returns.

The species stand in for the pseudopotentials of the paper's examples
(Sec. V.A uses Troullier-Martins / ONCV data that is not available here):
a Gaussian local potential V(r) = -v_amp exp(-r^2 / (2 v_sigma^2)) cut at
v_rcut and one s-type projector p(r) = exp(-r^2 / (2 p_sigma^2)) cut at
p_rcut with energy gamma, one electron per atom.

Cell dict keys
--------------
L (3 floats, Bohr), h (Bohr), fd_half_order (6 -> 12th order), pos
(n_atoms x 3 float64 in [0, L)), species (n_atoms int32), species_params
(list of dicts), n_electrons, rcut (Bohr), npl, kT (Ha), mu_mode
("solve" | "fixed"), mu (Ha, used when fixed), lanczos_steps.
"""

from __future__ import annotations

import numpy as np

GAUSS_SPECIES = dict(v_amp=2.0, v_sigma=0.8, v_rcut=4.8,
                     p_sigma=0.6, p_rcut=3.6, gamma=1.0, z_val=1.0)


def random_positions(rng: np.random.Generator, n_atoms: int, L, d_min: float,
                     max_tries: int = 200000) -> np.ndarray:
    """Random sequential addition: uniform in [0, L)^3, rejecting a candidate
    whose minimum-image distance to an accepted atom is below d_min."""
    L = np.asarray(L, dtype=np.float64)
    pos = np.empty((0, 3))
    tries = 0
    while pos.shape[0] < n_atoms:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms at this density")
        p = rng.uniform(0.0, 1.0, 3) * L
        if pos.shape[0]:
            d = pos - p
            d -= L * np.round(d / L)
            if np.min(np.einsum("ij,ij->i", d, d)) < d_min * d_min:
                continue
        pos = np.vstack([pos, p])
    return pos


def make_cell(L, h, pos, rcut, npl, kT, species=None, species_params=None,
              fd_half_order=6, n_electrons=None, mu_mode="solve", mu=0.0,
              lanczos_steps=20) -> dict:
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    if np.isscalar(L):
        L = (float(L),) * 3
    if species is None:
        species = np.zeros(pos.shape[0], dtype=np.int32)
    if species_params is None:
        species_params = [dict(GAUSS_SPECIES)]
    if n_electrons is None:
        n_electrons = float(sum(species_params[s]["z_val"] for s in species))
    return dict(L=tuple(float(x) for x in L), h=float(h),
                fd_half_order=int(fd_half_order), pos=pos,
                species=np.ascontiguousarray(species, dtype=np.int32),
                species_params=[dict(s) for s in species_params],
                n_electrons=float(n_electrons), rcut=float(rcut), npl=int(npl),
                kT=float(kT), mu_mode=mu_mode, mu=float(mu),
                lanczos_steps=int(lanczos_steps))


def random_cell(seed, L, h, n_atoms, d_min, rcut, npl, kT, **kw) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = random_positions(rng, n_atoms, (L, L, L) if np.isscalar(L) else L, d_min)
    return make_cell(L, h, pos, rcut, npl, kT, **kw)


# ----------------------------------------------------------------------------
# The five workloads.  Shapes follow the paper's high-temperature examples
# (Sec. V.A: a few tens of atoms per periodic cell, 12th-order FD, Chebyshev
# degree in the tens, truncation radius of a few Bohr), at synthetic species.
# ----------------------------------------------------------------------------

def tiny_cell(**kw) -> dict:
    """6 Bohr cube, h = 0.5 (12^3 nodes), 2 atoms (min spacing 2), R_cut = 2
    (9^3 cube), degree 24, kT = 0.1 Ha.  Small enough for dense diagonalisation."""
    args = dict(seed=0, L=6.0, h=0.5, n_atoms=2, d_min=2.0, rcut=2.0, npl=24, kT=0.1)
    args.update(kw)
    return random_cell(**args)


def fp64_cell(**kw) -> dict:
    """16 Bohr cube, h = 0.4 (40^3 = 64000 nodes), 64 atoms (min spacing 1.5),
    R_cut = 4 (21^3 cube), degree 60, kT = 0.05 Ha."""
    args = dict(seed=1, L=16.0, h=0.4, n_atoms=64, d_min=1.5, rcut=4.0, npl=60, kT=0.05)
    args.update(kw)
    return random_cell(**args)


def mixed_sweep_cells(degrees=(40, 60, 80)) -> list:
    """The 64000-node cell at several Chebyshev degrees (same positions)."""
    return [fp64_cell(npl=d) for d in degrees]


def batched_cells(n_cells=32, seed=3) -> list:
    """Independent uneven periodic cells drawn from one stream: n in {25..40}
    nodes per side at h = 0.4 (cell side 10-16 Bohr), 8-64 atoms (min spacing
    1.5), R_cut uniform in [3, 4], degree uniform in {30..80}, kT uniform in
    [0.03, 0.2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cells = []
    for _ in range(n_cells):
        n = int(rng.integers(25, 41))
        L = 0.4 * n
        n_atoms = int(rng.integers(8, 65))
        rcut = float(rng.uniform(3.0, 4.0))
        npl = int(rng.integers(30, 81))
        kT = float(rng.uniform(0.03, 0.2))
        pos = random_positions(rng, n_atoms, (L, L, L), 1.5)
        cells.append(make_cell(L, 0.4, pos, rcut, npl, kT))
    return cells


def large_cell(**kw) -> dict:
    """32 Bohr cube, h = 0.4 (80^3 = 512000 nodes), 512 atoms (min spacing
    1.5), R_cut = 5 (25^3 cube), degree 80, kT = 0.05 Ha."""
    args = dict(seed=4, L=32.0, h=0.4, n_atoms=512, d_min=1.5, rcut=5.0, npl=80, kT=0.05)
    args.update(kw)
    return random_cell(**args)


def node_sample(n_nodes_total: int, count: int, seed: int = 40) -> np.ndarray:
    """Sorted sample of distinct node indices (used for sampled comparisons)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_nodes_total, size=min(count, n_nodes_total), replace=False)).astype(np.int64)
