"""Writes scf_si35_oracle.json: the oracle's FP64 SCF on the 0.55 nm cluster
(Si35H36, geometry seed 1001, the model pseudopotential of the workloads,
h = 0.7 bohr, degree 10, 128 states, the oracle's Anderson mixing) run to
SRE < 1e-8 Ry.  Its occupied eigenvalues and Harris-Foulkes energy are the
reference that the device SCFs (FP64 and mixed precision), converged on
their own, are compared with.  Calls only oracle/ and the input generators
in synth/.

    python -m tests.golden.make_scf_si35
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import grid as G  # noqa: E402
from oracle import hamiltonian as OH  # noqa: E402
from oracle import scf as OS  # noqa: E402
from synth.cluster import make_cluster, n_states, random_block  # noqa: E402
from synth.workloads import MODEL_PP  # noqa: E402

SRE_TOL = 1e-8


def main():
    c = make_cluster(5.5, 1001)
    pp = OH.PseudoParams(**dataclasses.asdict(MODEL_PP))
    g = G.build_grid(c.domain_radius(), 0.7)
    nbr = G.neighbour_table(g)
    H = OH.build_hamiltonian(g, c.pos, c.species, pp)
    ne = c.n_electrons
    M = n_states(ne)
    e_ii = OS.ion_energy(c.pos, pp.charges(c.species))
    st = OS.ScfState(OS.sad_density(g, c.pos, c.species, ne), random_block(g.n, M, 2001), np.zeros(g.n))
    v0 = random_block(g.n, 1, 3001)[:, 0]
    t0 = time.time()
    for _ in range(200):
        r = OS.scf_step(H, nbr, st, ne, 10, v0, e_ii)
        print(f"step {r.step}: SRE {r.sre_ry:.3e} Ry, E {r.energy:.10f} Ha ({time.time() - t0:.0f} s)", flush=True)
        if r.sre_ry < SRE_TOL:
            break
    else:
        raise SystemExit("the oracle SCF did not reach the threshold")
    n_occ = ne // 2
    out = {"cluster": {"radius_angstrom": 5.5, "geometry_seed": 1001, "n_si": int(c.n_si), "n_h": int(c.n_h),
                       "n_atoms": int(c.n_atoms), "n_electrons": int(ne)},
           "h_bohr": 0.7, "degree": 10, "states": int(M), "steps": int(r.step), "sre_ry": float(r.sre_ry),
           "energy_ha": float(r.energy), "eig_occ_ha": [float(x) for x in r.eig[:n_occ]],
           "homo_ha": float(r.homo), "lumo_ha": float(r.lumo)}
    with open(os.path.join(HERE, "scf_si35_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "eig_occ_ha"}))


if __name__ == "__main__":
    main()
