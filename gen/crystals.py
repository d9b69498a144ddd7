"""Seeded synthetic structures and force constants.

Block conventions (shared input format, no method arithmetic here):

* fc2 block ``(i, j, R)`` holds the 3x3 matrix d^2E / du_(i,0) du_(j,R): atom ``i``
  sits in the home cell, atom ``j`` in the cell translated by the integer lattice
  vector ``R`` (Cartesian offset ``R @ cell``).
* fc3 block ``(i, j, R1, l, R2)`` holds the 3x3x3 tensor
  d^3E / du_(i,0) du_(j,R1) du_(l,R2).

Blocks with the same key are summed before they are returned, so every key
appears once.  ``cell`` rows are the lattice vectors.

Generators:

* Keating valence force field (bond-stretch + bond-bend) for diamond-like
  networks.  The Hessian is assembled as sum 2c grad(f) grad(f)^T at the given
  geometry, i.e. the geometry is taken as the reference one; this makes fc2
  positive semi-definite and translation invariant by construction.
* Central pair springs k(r) with rest length equal to the actual distance, for
  random cells.
* Random third-order constants: every pair and triangle of sites whose pairwise
  distances are all within ``rc3`` gets, once per lattice-translation orbit, a
  Gaussian tensor over its 3c coordinates that is symmetrised over the index
  permutations and projected onto the complement of rigid translations on all
  three indices.  The sum over orbits and translations is therefore
  permutation symmetric, periodic and satisfies the acoustic sum rule.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

SEED_BASE = 200901967
M_SI = 28.09
M_GE = 72.63

# Keating constants for silicon (common literature values), in eV/A^2:
# alpha = 48.5 N/m, beta = 13.8 N/m.
KEATING_ALPHA = 3.027
KEATING_BETA = 0.861


@dataclass
class Crystal:
    name: str
    cell: np.ndarray            # (3, 3) rows = lattice vectors [A]
    positions: np.ndarray       # (N, 3) Cartesian [A]
    masses: np.ndarray          # (N,) [amu]
    fc2_i: np.ndarray           # (nb2,) int32
    fc2_j: np.ndarray           # (nb2,) int32
    fc2_R: np.ndarray           # (nb2, 3) int32
    fc2_val: np.ndarray         # (nb2, 3, 3) float64 [eV/A^2]
    fc3_i: np.ndarray           # (nb3,) int32
    fc3_j: np.ndarray           # (nb3,) int32
    fc3_l: np.ndarray           # (nb3,) int32
    fc3_R1: np.ndarray          # (nb3, 3) int32
    fc3_R2: np.ndarray          # (nb3, 3) int32
    fc3_val: np.ndarray         # (nb3, 3, 3, 3) float64 [eV/A^3]
    grid: Tuple[int, int, int] = (1, 1, 1)
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def n_modes(self) -> int:
        return 3 * self.n_atoms

    @property
    def n_k(self) -> int:
        return int(np.prod(self.grid))

    def with_fc3_scaled(self, s: float) -> "Crystal":
        c = _copy(self)
        c.fc3_val = self.fc3_val * s
        return c

    def with_grid(self, grid) -> "Crystal":
        c = _copy(self)
        c.grid = tuple(int(g) for g in grid)
        return c


def _copy(c: Crystal) -> Crystal:
    return Crystal(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                      for k, v in c.__dict__.items()})


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _translations(cell: np.ndarray, rcut: float) -> np.ndarray:
    """Integer translations that can bring an image within ``rcut`` of any
    site of a wrapped cell."""
    B = np.linalg.inv(cell).T             # rows: reciprocal vectors b_i, a_i.b_j = delta
    heights = 1.0 / np.linalg.norm(B, axis=1)
    nr = np.ceil(rcut / heights).astype(int) + 1
    rng = [np.arange(-m, m + 1) for m in nr]
    return np.array(list(itertools.product(*rng)), dtype=np.int64)


def neighbour_lists(cell, pos, rcut) -> List[List[Tuple[int, Tuple[int, int, int], float]]]:
    """For each home atom i: [(j, R, distance)] with 0 < distance <= rcut."""
    Rs = _translations(cell, rcut)
    Rc = Rs @ cell
    out = []
    n = pos.shape[0]
    for i in range(n):
        disp = pos[None, :, :] + Rc[:, None, :] - pos[i][None, None, :]   # (nR, n, 3)
        d = np.linalg.norm(disp, axis=2)
        rr, jj = np.nonzero((d <= rcut) & (d > 1e-8))
        lst = [(int(j), tuple(int(x) for x in Rs[r]), float(d[r, j])) for r, j in zip(rr, jj)]
        lst.sort()
        out.append(lst)
    return out


def _site_pos(cell, pos, site):
    a, R = site
    return pos[a] + np.asarray(R, dtype=float) @ cell


def _canonical(sites: Sequence[Tuple[int, Tuple[int, int, int]]]):
    best = None
    for a, Ra in sites:
        key = tuple(sorted((b, (Rb[0] - Ra[0], Rb[1] - Ra[1], Rb[2] - Ra[2])) for b, Rb in sites))
        if best is None or key < best:
            best = key
    return best


def _sub(R1, R2):
    return (R1[0] - R2[0], R1[1] - R2[1], R1[2] - R2[2])


# ----------------------------------------------------------------------------
# fc2 generators
# ----------------------------------------------------------------------------

def _accumulate_terms_fc2(terms) -> Dict:
    """terms: iterable of (c, [(site, g)]) representing E += c f^2 with
    grad f = g at each site; adds 2 c g_a g_b^T to block (a home; b)."""
    acc: Dict = {}
    for c, sg in terms:
        for (sa, ga) in sg:
            for (sb, gb) in sg:
                key = (sa[0], sb[0], _sub(sb[1], sa[1]))
                blk = 2.0 * c * np.outer(ga, gb)
                if key in acc:
                    acc[key] += blk
                else:
                    acc[key] = blk
    return acc


def _fc2_arrays(acc: Dict):
    keys = sorted(acc.keys())
    i = np.array([k[0] for k in keys], dtype=np.int32)
    j = np.array([k[1] for k in keys], dtype=np.int32)
    R = np.array([k[2] for k in keys], dtype=np.int32).reshape(-1, 3)
    val = np.array([acc[k] for k in keys], dtype=np.float64).reshape(-1, 3, 3)
    return i, j, R, val


def keating_fc2(cell, pos, bonds_of, d0, alpha=KEATING_ALPHA, beta=KEATING_BETA):
    """Keating fc2 at the given geometry.

    ``bonds_of[i]`` lists the bonded neighbours (j, R) of home atom i.  Bond
    stretching is counted from both ends of a bond (Keating's original sum),
    angle bending once per centre and unordered neighbour pair."""
    cb = 3.0 * alpha / (16.0 * d0 * d0)
    ca = 3.0 * beta / (8.0 * d0 * d0)
    terms = []
    zero = (0, 0, 0)
    for i, nbrs in enumerate(bonds_of):
        xi = pos[i]
        vecs = [(_site_pos(cell, pos, (j, R)) - xi, (j, R)) for (j, R) in nbrs]
        for r, sj in vecs:
            terms.append((cb, [((i, zero), -2.0 * r), (sj, 2.0 * r)]))
        for (r1, s1), (r2, s2) in itertools.combinations(vecs, 2):
            terms.append((ca, [((i, zero), -(r1 + r2)), (s1, r2), (s2, r1)]))
    return _fc2_arrays(_accumulate_terms_fc2(terms))


def spring_constant(r):
    """Central spring constant [eV/A^2] used for random cells."""
    return 8.0 * np.exp(-(r - 2.35) / 0.6)


def pair_spring_fc2(cell, pos, rc2):
    nl = neighbour_lists(cell, pos, rc2)
    seen = set()
    terms = []
    zero = (0, 0, 0)
    for i, lst in enumerate(nl):
        for (j, R, d) in lst:
            key = _canonical([(i, zero), (j, R)])
            if key in seen:
                continue
            seen.add(key)
            u = (_site_pos(cell, pos, (j, R)) - pos[i]) / d
            c = 0.5 * spring_constant(d)
            terms.append((c, [((i, zero), -u), ((j, R), u)]))
    return _fc2_arrays(_accumulate_terms_fc2(terms))


# ----------------------------------------------------------------------------
# fc3 generator
# ----------------------------------------------------------------------------

def cluster_orbits(cell, pos, rc3):
    """Pair and triangle clusters with all pairwise distances <= rc3, one
    representative per translation orbit, in canonical sorted order."""
    nl = neighbour_lists(cell, pos, rc3)
    zero = (0, 0, 0)
    orbits = {}
    for i, lst in enumerate(nl):
        home = (i, zero)
        sites = [(j, R) for (j, R, _) in lst]
        for s in sites:
            key = _canonical([home, s])
            orbits.setdefault(key, key)
        spos = [_site_pos(cell, pos, s) for s in sites]
        for a in range(len(sites)):
            for b in range(a + 1, len(sites)):
                if np.linalg.norm(spos[a] - spos[b]) <= rc3 + 1e-12:
                    key = _canonical([home, sites[a], sites[b]])
                    orbits.setdefault(key, key)
    return sorted(orbits.keys())


def _translation_projector(c: int) -> np.ndarray:
    P = np.zeros((3 * c, 3 * c))
    for a in range(c):
        for b in range(c):
            P[3 * a:3 * a + 3, 3 * b:3 * b + 3] = np.eye(3) / c
    return np.eye(3 * c) - P


def random_fc3(cell, pos, rc3, rng, sigma=1.0):
    orbits = cluster_orbits(cell, pos, rc3)
    acc: Dict = {}
    perms = list(itertools.permutations(range(3)))
    for orb in orbits:
        c = len(orb)
        T = rng.normal(0.0, sigma, size=(3 * c,) * 3)
        T = sum(np.transpose(T, p) for p in perms) / 6.0
        Q = _translation_projector(c)
        T = np.einsum('ia,jb,kc,abc->ijk', Q, Q, Q, T, optimize=True)
        for a in range(c):
            for b in range(c):
                for d in range(c):
                    sa, sb, sd = orb[a], orb[b], orb[d]
                    key = (sa[0], sb[0], _sub(sb[1], sa[1]), sd[0], _sub(sd[1], sa[1]))
                    blk = T[3 * a:3 * a + 3, 3 * b:3 * b + 3, 3 * d:3 * d + 3]
                    if key in acc:
                        acc[key] = acc[key] + blk
                    else:
                        acc[key] = blk.copy()
    keys = sorted(acc.keys())
    i = np.array([k[0] for k in keys], dtype=np.int32)
    j = np.array([k[1] for k in keys], dtype=np.int32)
    R1 = np.array([k[2] for k in keys], dtype=np.int32).reshape(-1, 3)
    l = np.array([k[3] for k in keys], dtype=np.int32)
    R2 = np.array([k[4] for k in keys], dtype=np.int32).reshape(-1, 3)
    val = np.array([acc[k] for k in keys], dtype=np.float64).reshape(-1, 3, 3, 3)
    return i, j, l, R1, R2, val, len(orbits)


# ----------------------------------------------------------------------------
# structures
# ----------------------------------------------------------------------------

def _make(name, cell, pos, masses, fc2, fc3, grid, meta):
    i2, j2, R2_, v2 = fc2
    i3, j3, l3, R1, R2, v3, norb = fc3
    meta = dict(meta)
    meta['fc3_orbits'] = norb
    return Crystal(name=name, cell=np.asarray(cell, float), positions=np.asarray(pos, float),
                   masses=np.asarray(masses, float),
                   fc2_i=i2, fc2_j=j2, fc2_R=R2_, fc2_val=v2,
                   fc3_i=i3, fc3_j=j3, fc3_l=l3, fc3_R1=R1, fc3_R2=R2, fc3_val=v3,
                   grid=tuple(int(g) for g in grid), meta=meta)


def diamond_si(grid=(4, 4, 4), rc3=2.6, a=5.43, seed=SEED_BASE + 0, masses=(M_SI, M_SI),
               sigma3=1.0):
    """Two-atom primitive diamond cell with Keating fc2 and random fc3."""
    cell = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    pos = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
    d0 = a * np.sqrt(3.0) / 4.0
    nl = neighbour_lists(cell, pos, 0.5 * (d0 + a / np.sqrt(2.0)))
    bonds_of = [[(j, R) for (j, R, _) in lst] for lst in nl]
    fc2 = keating_fc2(cell, pos, bonds_of, d0)
    rng = np.random.default_rng(seed)
    fc3 = random_fc3(cell, pos, rc3, rng, sigma=sigma3)
    return _make(f"si-diamond-2at-{grid[0]}x{grid[1]}x{grid[2]}-rc3_{rc3:g}", cell, pos,
                 np.asarray(masses, float), fc2, fc3, grid, {'rc3': rc3, 'seed': seed})


def _rsa_packing(n, L, dmin, rng, max_tries=200000):
    pts = np.zeros((0, 3))
    tries = 0
    while pts.shape[0] < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random packing failed")
        x = rng.uniform(0.0, L, size=3)
        if pts.shape[0]:
            d = pts - x
            d -= L * np.round(d / L)
            if np.min(np.linalg.norm(d, axis=1)) < dmin:
                continue
        pts = np.vstack([pts, x])
    return pts


def cage_cell(n_atoms=46, L=10.2, dmin=2.2, jitter=0.05, rc2=4.5, rc3=4.5, grid=(5, 5, 5),
              seed=SEED_BASE + 2):
    """Clathrate-like cubic cell: seeded min-distance packing, jittered, all Si."""
    rng = np.random.default_rng(seed)
    pos = _rsa_packing(n_atoms, L, dmin, rng)
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    pos = np.mod(pos, L)
    masses = np.full(n_atoms, M_SI)
    cell = np.eye(3) * L
    fc2 = pair_spring_fc2(cell, pos, rc2)
    fc3 = random_fc3(cell, pos, rc3, rng)
    return _make(f"cage-{n_atoms}at-{grid[0]}x{grid[1]}x{grid[2]}", cell, pos, masses, fc2, fc3,
                 grid, {'rc3': rc3, 'seed': seed, 'L': L})


def random_crystal(n_atoms, g, rng, vol_per_atom=20.0, dmin=2.2, rc=4.0, name=None):
    L = (vol_per_atom * n_atoms) ** (1.0 / 3.0)
    pos = _rsa_packing(n_atoms, L, dmin, rng)
    species = rng.integers(0, 2, size=n_atoms)
    masses = np.where(species == 0, M_SI, M_GE)
    cell = np.eye(3) * L
    fc2 = pair_spring_fc2(cell, pos, rc)
    fc3 = random_fc3(cell, pos, rc, rng)
    return _make(name or f"random-{n_atoms}at-{g}^3", cell, pos, masses, fc2, fc3, (g, g, g),
                 {'rc3': rc, 'L': L})


def batch_crystals(count=32, n_range=(2, 54), g_range=(4, 10), seed=SEED_BASE + 3):
    """Many crystals of uneven cell size and q-grid (one seeded stream)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        g = int(rng.integers(g_range[0], g_range[1] + 1))
        out.append(random_crystal(n, g, rng, name=f"batch{b:02d}-{n}at-{g}^3"))
    return out


def sige_supercell(reps=5, a=5.43, x_ge=0.5, jitter=0.1, rc3=4.0, seed=SEED_BASE + 4):
    """Disordered Si(1-x)Ge(x): reps^3 conventional diamond cells, jittered
    sites, Ge placed by a seeded permutation; Keating fc2 on the ideal bond graph
    evaluated at the jittered geometry; Gamma point only."""
    rng = np.random.default_rng(seed)
    basis = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0],
                      [1, 1, 1], [1, 3, 3], [3, 1, 3], [3, 3, 1]], dtype=float) / 4.0
    L = reps * a
    frac = []
    for c in itertools.product(range(reps), repeat=3):
        for b in basis:
            frac.append((np.asarray(c, float) + b) / reps)
    frac = np.array(frac)
    cell = np.eye(3) * L
    ideal = frac * L
    n = ideal.shape[0]
    d0 = a * np.sqrt(3.0) / 4.0
    nl = neighbour_lists(cell, ideal, 0.5 * (d0 + a / np.sqrt(2.0)))
    bonds_of = [[(j, R) for (j, R, _) in lst] for lst in nl]
    pos = ideal + rng.uniform(-jitter, jitter, size=ideal.shape)
    n_ge = int(round(x_ge * n))
    perm = rng.permutation(n)
    masses = np.full(n, M_SI)
    masses[perm[:n_ge]] = M_GE
    # Keep R offsets of the ideal bond graph; jittered positions stay unwrapped
    # so that the offsets remain valid.
    fc2 = keating_fc2(cell, pos, bonds_of, d0)
    fc3 = random_fc3(cell, pos, rc3, rng)
    return _make(f"sige-{n}at-gamma", cell, pos, masses, fc2, fc3, (1, 1, 1),
                 {'rc3': rc3, 'seed': seed, 'reps': reps})


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    # 2-atom diamond, 1st-shell fc3, 4^3, one temperature, FP64.
    'diamond-2at-4x4x4-shell1': dict(kind='diamond', grid=(4, 4, 4), rc3=2.6, T=(300.0,),
                                     sigma_thz=0.1),
    # same cell, fc3 to the 3rd shell, 16^3, three temperatures.
    'diamond-2at-16x16x16-shell3': dict(kind='diamond', grid=(16, 16, 16), rc3=4.7,
                                        T=(100.0, 300.0, 600.0), sigma_thz=0.1),
    # 46-atom clathrate-like cage cell, 5^3.
    'cage-46at-5x5x5': dict(kind='cage', grid=(5, 5, 5), rc3=4.5, T=(300.0,), sigma_thz=0.1),
    # 1000-atom SiGe, Gamma only.
    'sige-1000at-gamma': dict(kind='sige', reps=5, rc3=4.0, T=(300.0,), sigma_thz=0.1),
    # 64-atom SiGe, Gamma only (small version of the above for oracle parity).
    'sige-64at-gamma': dict(kind='sige', reps=2, rc3=4.0, T=(300.0,), sigma_thz=0.1),
}


def workload(name: str) -> Crystal:
    w = WORKLOADS[name]
    if w['kind'] == 'diamond':
        return diamond_si(grid=w['grid'], rc3=w['rc3'])
    if w['kind'] == 'cage':
        return cage_cell(grid=w['grid'], rc3=w['rc3'])
    if w['kind'] == 'sige':
        return sige_supercell(reps=w['reps'], rc3=w['rc3'])
    raise KeyError(name)
