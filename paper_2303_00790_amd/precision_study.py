"""Mixed precision against FP64 on one cluster (ChFSI with an FP32 filter and
FP32 Gram products, FP64 Cholesky, eigensolver, potentials and mixing,
against the all-FP64 SCF), run by the library's SCF to SRE < 1e-4 Ry from
the same start block.

    python -m paper_2303_00790_amd.precision_study --workload d3nm --out prec.json

Reports the converged energies, the largest eigenvalue difference over the
occupied states, the energy difference per atom, SCF step counts and the
time per SCF step of both runs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def run_one(cluster, pp, dtype: str, degree: int, log):
    import torch
    from . import scf as S
    st = S.setup(cluster, pp, dtype=dtype, degree=degree)
    H = st["H"]
    rho = H.sad_density(cluster.pos, cluster.species, cluster.n_electrons)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = S.run(st, rho, max_steps=80, sre_tol_ry=1e-4, log=log)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{dtype}: {res.steps} SCF steps, converged {res.converged}, E = {res.energy:.10f} Ha, {dt:.1f} s")
    out = dict(steps=res.steps, converged=res.converged, energy=res.energy, eig=np.asarray(res.eig), seconds=dt,
               n_points=H.n_points, M=st["M"])
    del st, H
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP, WORKLOADS

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="d3nm")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    wl = WORKLOADS[args.workload]

    def log(msg):
        print(msg, flush=True)

    c = make_cluster(wl.radius_angstrom, wl.geometry_seed, wl.sigma)
    r64 = run_one(c, MODEL_PP, "f64", wl.degree, log)
    r32 = run_one(c, MODEL_PP, "f32", wl.degree, log)
    n_occ = c.n_electrons // 2
    d_eig = np.abs(r32["eig"][:n_occ] - r64["eig"][:n_occ])
    res = dict(workload=wl.name, n_si=c.n_si, n_h=c.n_h, n_points=r64["n_points"], states=r64["M"], degree=wl.degree,
               energy_f64=r64["energy"], energy_mixed=r32["energy"],
               de_per_atom_ha=abs(r32["energy"] - r64["energy"]) / c.n_atoms,
               max_occ_eig_diff_ha=float(d_eig.max()), mean_occ_eig_diff_ha=float(d_eig.mean()),
               steps_f64=r64["steps"], steps_mixed=r32["steps"],
               s_per_step_f64=r64["seconds"] / r64["steps"], s_per_step_mixed=r32["seconds"] / r32["steps"],
               converged=bool(r64["converged"] and r32["converged"]))
    log(json.dumps(res))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()
