"""Small oracle systems shared by the CPU pin tests, built once per process.

The returned objects are shared between test modules and must be treated
as read-only."""
import functools
import math

import numpy as np

from oracle import grid as G
from oracle import hamiltonian as OH
from oracle import scf as S
from synth.cluster import BOHR_ANGSTROM, random_block

# SiH4: Si at the origin, H at 1.48 Angstrom along the four tetrahedral bonds
_D = 1.48 / BOHR_ANGSTROM / math.sqrt(3)
H_POS = [[0, 0, 0], [_D, _D, _D], [_D, -_D, -_D], [-_D, _D, -_D], [-_D, -_D, _D]]


@functools.lru_cache(maxsize=None)
def tiny():
    """Two Si and one H on a 6 bohr sphere at h = 0.8, with the dense H and
    its exact eigenpairs: (H, H_dense, eigenvalues, eigenvectors)."""
    pos = np.array([[0.2, -0.3, 0.1], [2.4, 2.1, -2.2], [-1.6, 1.2, 1.4]])
    species = np.array([0, 0, 1], np.int32)
    g = G.build_grid(6.0, 0.8)
    H = OH.build_hamiltonian(g, pos, species, OH.PseudoParams(h_s=2.0, h_p=0.5))
    Hd = H.dense()
    lam, V = np.linalg.eigh(Hd)
    return H, Hd, lam, V


@functools.lru_cache(maxsize=None)
def sih4_scf():
    """30 oracle SCF steps of SiH4 from the superposed atomic density:
    (H, neighbour table, final state, step reports)."""
    pos = np.array(H_POS)
    species = np.array([0, 1, 1, 1, 1], np.int32)
    g = G.build_grid(float(np.sqrt((pos ** 2).sum(1)).max()) + 5.0, 0.7)
    nbr = G.neighbour_table(g)
    pp = OH.PseudoParams()
    H = OH.build_hamiltonian(g, pos, species, pp)
    st = S.ScfState(S.sad_density(g, pos, species, 8), random_block(g.n, 10, 5), np.zeros(g.n))
    eii = S.ion_energy(pos, pp.charges(species))
    reps = [S.scf_step(H, nbr, st, 8, 12, random_block(g.n, 1, 6)[:, 0], eii) for _ in range(30)]
    return H, nbr, st, reps
