"""Test helper: fold a crystal into its grid supercell (real space).

The supercell of a crystal over a Gamma-centred grid G holds N_k = G1 G2 G3
copies of the unit cell; force-constant blocks are re-indexed onto supercell
atoms and supercell lattice vectors.  Used by tests that compare the Bloch
(crystal) formulation against plain real-space sums on the supercell.
"""

import itertools
from collections import defaultdict

import numpy as np

from gen.crystals import Crystal


def cells(grid):
    return [tuple(L) for L in itertools.product(range(grid[0]), range(grid[1]), range(grid[2]))]


def cell_index(L, grid):
    return (L[0] * grid[1] + L[1]) * grid[2] + L[2]


def fold(crystal, grid=None) -> Crystal:
    g = tuple(crystal.grid if grid is None else grid)
    N = crystal.n_atoms
    G = np.asarray(g)
    Ls = cells(g)

    def site(L, a, R):
        tot = np.asarray(L) + np.asarray(R)
        lp = tuple(int(x) for x in np.mod(tot, G))
        Rs = tuple(int(x) for x in np.floor_divide(tot, G))
        return cell_index(lp, g) * N + int(a), Rs

    acc2 = defaultdict(lambda: np.zeros((3, 3)))
    for L in Ls:
        home = cell_index(L, g) * N
        for i, j, R, v in zip(crystal.fc2_i, crystal.fc2_j, crystal.fc2_R, crystal.fc2_val):
            B, Rs = site(L, j, R)
            acc2[(home + int(i), B, Rs)] += v
    acc3 = defaultdict(lambda: np.zeros((3, 3, 3)))
    for L in Ls:
        home = cell_index(L, g) * N
        for i, j, l, R1, R2, v in zip(crystal.fc3_i, crystal.fc3_j, crystal.fc3_l,
                                      crystal.fc3_R1, crystal.fc3_R2, crystal.fc3_val):
            B, R1s = site(L, j, R1)
            C, R2s = site(L, l, R2)
            acc3[(home + int(i), B, R1s, C, R2s)] += v
    k2 = sorted(acc2)
    k3 = sorted(acc3)
    pos = np.array([crystal.positions[a] + np.asarray(L, float) @ crystal.cell
                    for L in Ls for a in range(N)])
    masses = np.array([crystal.masses[a] for L in Ls for a in range(N)])
    return Crystal(
        name=crystal.name + "-folded", cell=crystal.cell * G[:, None], positions=pos,
        masses=masses,
        fc2_i=np.array([k[0] for k in k2], np.int32), fc2_j=np.array([k[1] for k in k2], np.int32),
        fc2_R=np.array([k[2] for k in k2], np.int32).reshape(-1, 3),
        fc2_val=np.array([acc2[k] for k in k2]).reshape(-1, 3, 3),
        fc3_i=np.array([k[0] for k in k3], np.int32), fc3_j=np.array([k[1] for k in k3], np.int32),
        fc3_l=np.array([k[3] for k in k3], np.int32),
        fc3_R1=np.array([k[2] for k in k3], np.int32).reshape(-1, 3),
        fc3_R2=np.array([k[4] for k in k3], np.int32).reshape(-1, 3),
        fc3_val=np.array([acc3[k] for k in k3]).reshape(-1, 3, 3, 3),
        grid=(1, 1, 1), meta={'folded_from': crystal.name, 'grid': g})


def dense_fc2(sc: Crystal) -> np.ndarray:
    """Real-space Hessian of a (super)cell treated as an isolated periodic box
    (all images summed), shape (3N, 3N) in eV/A^2."""
    n = sc.n_modes
    H = np.zeros((n, n))
    for i, j, v in zip(sc.fc2_i, sc.fc2_j, sc.fc2_val):
        H[3 * i:3 * i + 3, 3 * j:3 * j + 3] += v
    return H


def dense_fc3(sc: Crystal) -> np.ndarray:
    n = sc.n_modes
    T = np.zeros((n, n, n))
    for i, j, l, v in zip(sc.fc3_i, sc.fc3_j, sc.fc3_l, sc.fc3_val):
        T[3 * i:3 * i + 3, 3 * j:3 * j + 3, 3 * l:3 * l + 3] += v
    return T
