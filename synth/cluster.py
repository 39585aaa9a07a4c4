"""Seeded synthetic inputs: hydrogen-passivated silicon nanoclusters.

This module only builds inputs (atom positions, species, random blocks).  It
holds none of the eigensolver's arithmetic and is the single piece of code
that both the product path and the test oracle may use.

Cluster rule (the paper's system description: spherical Si nanoclusters cut
from the diamond structure, surface dangling bonds passivated by H):

* diamond lattice of constant ``a``, origin on an atom (atom-centred sphere);
* keep every Si with ``|r| <= R``;
* repeatedly drop Si that have fewer than two Si nearest neighbours until no
  more are dropped (a fixpoint);
* put one H at ``d_SiH`` along every tetrahedral bond of a kept Si whose
  partner is missing;
* finally perturb every coordinate of every atom by N(0, sigma^2) drawn from
  ``numpy.random.default_rng(seed)``; neighbour decisions and the cluster
  radius use the unperturbed positions.

Lattice sites are handled in exact integer coordinates in units of a/4:
sublattice A has all-even coordinates with a sum divisible by 4, sublattice B
is A shifted by (1, 1, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BOHR_ANGSTROM = 0.529177210903  # 1 bohr in angstrom
A_SI_OBSERVED = 5.43            # angstrom, observed lattice constant
A_SI_OPTIMISED = 5.38           # angstrom, the paper's LDA-optimised value
D_SIH = 1.48                    # angstrom, Si-H bond length
SPECIES_SI, SPECIES_H = 0, 1

# The four tetrahedral bond directions of a sublattice-A atom, in units of
# a/4; a sublattice-B atom bonds along the negated directions.
_BONDS_A = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.int64)


@dataclass
class Cluster:
    pos: np.ndarray        # [n_atoms, 3] float64, bohr, perturbed
    pos0: np.ndarray       # [n_atoms, 3] float64, bohr, unperturbed
    species: np.ndarray    # [n_atoms] int32, 0 = Si, 1 = H
    n_si: int
    n_h: int

    @property
    def n_atoms(self) -> int:
        return int(self.species.size)

    @property
    def n_electrons(self) -> int:
        return 4 * self.n_si + self.n_h

    @property
    def r_cluster(self) -> float:
        """Largest distance of an unperturbed atom from the centre atom, bohr."""
        p = self.pos0
        return float(np.max(np.sqrt(p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1] + p[:, 2] * p[:, 2])))

    def domain_radius(self, margin_bohr: float = 6.0) -> float:
        return self.r_cluster + margin_bohr


def _lattice_si(radius_over_a: float) -> np.ndarray:
    """Integer (a/4 units) diamond sites with |r| <= R, sorted lexicographically."""
    lim = int(math.floor(4.0 * radius_over_a)) + 1
    r2max = (4.0 * radius_over_a) ** 2
    g = np.arange(-lim, lim + 1, dtype=np.int64)
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    even = (x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0) & ((x + y + z) % 4 == 0)
    odd = (x % 2 == 1) & (y % 2 == 1) & (z % 2 == 1) & ((x + y + z) % 4 == 3)
    keep = (even | odd) & ((x * x + y * y + z * z).astype(np.float64) <= r2max)
    return np.stack([x[keep], y[keep], z[keep]], axis=1)


def _bond_dirs(site: np.ndarray) -> np.ndarray:
    return _BONDS_A if site[0] % 2 == 0 else -_BONDS_A


def silicon_cluster_counts(radius_over_a: float) -> tuple[np.ndarray, list[tuple[np.ndarray, np.ndarray]]]:
    """Pruned Si sites (integer, a/4 units) and their dangling bonds."""
    si = _lattice_si(radius_over_a)
    present = {tuple(s) for s in si.tolist()}
    while True:
        drop = []
        for s in present:
            d = _BONDS_A if s[0] % 2 == 0 else -_BONDS_A
            nn = sum((s[0] + b[0], s[1] + b[1], s[2] + b[2]) in present for b in d)
            if nn < 2:
                drop.append(s)
        if not drop:
            break
        for s in drop:
            present.discard(s)
    kept = np.array(sorted(present), dtype=np.int64).reshape(-1, 3)
    dangling = []
    for s in kept:
        for b in _bond_dirs(s):
            if (s[0] + b[0], s[1] + b[1], s[2] + b[2]) not in present:
                dangling.append((s, b))
    return kept, dangling


def make_cluster(radius_angstrom: float, seed: int, sigma_angstrom: float = 0.02,
                 a_angstrom: float = A_SI_OBSERVED, d_sih: float = D_SIH) -> Cluster:
    """Build the seeded, perturbed Si/H cluster of the given radius (angstrom)."""
    si, dangling = silicon_cluster_counts(radius_angstrom / a_angstrom)
    q = a_angstrom / 4.0
    si_pos = si.astype(np.float64) * q
    h_pos = np.array([s.astype(np.float64) * q + d_sih * b / math.sqrt(3.0) for s, b in dangling],
                     dtype=np.float64).reshape(-1, 3)
    pos0 = np.concatenate([si_pos, h_pos], axis=0)
    species = np.concatenate([np.full(len(si_pos), SPECIES_SI, np.int32),
                              np.full(len(h_pos), SPECIES_H, np.int32)])
    rng = np.random.default_rng(seed)
    pos = pos0 + rng.normal(0.0, sigma_angstrom, size=pos0.shape) if sigma_angstrom > 0 else pos0.copy()
    return Cluster(pos=pos / BOHR_ANGSTROM, pos0=pos0 / BOHR_ANGSTROM, species=species,
                   n_si=len(si_pos), n_h=len(h_pos))


def random_block(n_rows: int, n_vec: int, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) block [n_rows, n_vec], float64, from default_rng(seed)."""
    return np.random.default_rng(seed).standard_normal((n_rows, n_vec))


def n_states(n_electrons: int, extra: float = 0.10, multiple: int = 64) -> int:
    """Number of states: occupied count plus ``extra``, rounded up to ``multiple``."""
    occ = n_electrons // 2
    m = int(math.ceil((1.0 + extra) * occ - 1e-12))
    return ((m + multiple - 1) // multiple) * multiple
