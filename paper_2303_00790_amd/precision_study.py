"""Mixed precision against FP64 on one cluster (ChFSI with an FP32 filter and
FP32 Gram products, FP64 Cholesky, eigensolver, potentials and mixing,
against the all-FP64 SCF), both run by the library's SCF from the same start
block to the same SRE threshold.

    python -m paper_2303_00790_amd.precision_study --workload d3nm --out prec.json
    python -m paper_2303_00790_amd.precision_study --workload d5nm --only f64 --sre-tol 1e-5 --out f64.json
    python -m paper_2303_00790_amd.precision_study --combine f64.json f32.json --out prec.json
    python -m paper_2303_00790_amd.precision_study --workload d5nm --only f32 --sre-tol 1e-3 --rho-out rho1.npy
    python -m paper_2303_00790_amd.precision_study --workload d5nm --only f64 --sre-tol 1e-5 --rho-in rho1.npy

Reports the converged energies, the largest eigenvalue difference over the
occupied states, the energy difference per atom, SCF step counts and the
time per SCF step of both runs.  --only runs one precision and writes its
record (energy, occupied eigenvalues, steps, times); --combine compares two
such records (so the two runs can take separate sessions on the device).
--rho-out / --rho-in save and restart from a mixed input density, so that a
long SCF can be split: both precisions then converge from the same density
(and the same start vectors) to their own fixed points.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def run_one(cluster, pp, dtype: str, degree: int, log, sre_tol: float = 1e-4, max_steps: int = 80,
            trace=None, rho_in=None, rho_out=None):
    """One SCF from the superposition start, or from the density in rho_in
    (.npy of the inside-point values in curve order); rho_out (optional
    path) receives the last mixed input density in the same form."""
    import torch
    from . import scf as S
    t0 = time.perf_counter()
    st = S.setup(cluster, pp, dtype=dtype, degree=degree)
    H = st["H"]
    if rho_in:
        rho = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
        rho[st["rows"]] = torch.from_numpy(np.load(rho_in)).cuda()
        log(f"{dtype}: start density from {os.path.basename(rho_in)}")
    else:
        rho = H.sad_density(cluster.pos, cluster.species, cluster.n_electrons)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log(f"{dtype}: setup {t_setup:.1f} s, {H.n_points} points, {st['M']} states, work block {st['W'].shape[1]} columns")
    t0 = time.perf_counter()
    res = S.run(st, rho, max_steps=max_steps, sre_tol_ry=sre_tol, log=log, trace=trace)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{dtype}: {res.steps} SCF steps, converged {res.converged}, E = {res.energy:.10f} Ha, {dt:.1f} s")
    if rho_out:
        rho_last = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
        st["scf"].fields(rho_last)
        np.save(rho_out, rho_last[st["rows"]].cpu().numpy())
    n_occ = cluster.n_electrons // 2
    out = dict(dtype=dtype, steps=res.steps, converged=bool(res.converged), energy=res.energy,
               eig_occ=[float(x) for x in np.asarray(res.eig)[:n_occ]], seconds=dt, setup_s=t_setup,
               n_points=H.n_points, M=st["M"], sre_last=res.reports[-1]["sre_ry"], sre_tol=sre_tol,
               step_seconds=[r["seconds"] for r in res.reports])
    del st, H
    torch.cuda.empty_cache()
    return out


def compare(c_info: dict, r64: dict, r32: dict) -> dict:
    e64, e32 = np.asarray(r64["eig_occ"]), np.asarray(r32["eig_occ"])
    d_eig = np.abs(e32 - e64)
    return dict(c_info, n_points=r64["n_points"], states=r64["M"],
                energy_f64=r64["energy"], energy_mixed=r32["energy"],
                de_per_atom_ha=abs(r32["energy"] - r64["energy"]) / c_info["n_atoms"],
                max_occ_eig_diff_ha=float(d_eig.max()), mean_occ_eig_diff_ha=float(d_eig.mean()),
                steps_f64=r64["steps"], steps_mixed=r32["steps"], sre_tol_ry=r64["sre_tol"],
                sre_last_f64=r64["sre_last"], sre_last_mixed=r32["sre_last"],
                s_per_step_f64=r64["seconds"] / r64["steps"], s_per_step_mixed=r32["seconds"] / r32["steps"],
                start_density_f64=r64.get("start_density", "superposition"),
                start_density_mixed=r32.get("start_density", "superposition"),
                converged=bool(r64["converged"] and r32["converged"]))


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--workload", default="d3nm")
    ap.add_argument("--only", choices=["f64", "f32"], default=None)
    ap.add_argument("--sre-tol", type=float, default=1e-4, help="SRE threshold (Ry) of both runs")
    ap.add_argument("--max-steps", type=int, default=80)
    ap.add_argument("--trace", default=None, help="JSON lines, one per SCF step")
    ap.add_argument("--combine", nargs=2, metavar=("F64_JSON", "F32_JSON"), default=None)
    ap.add_argument("--rho-in", default=None, help="start density (.npy, inside points in curve order)")
    ap.add_argument("--rho-out", default=None, help="save the last mixed input density (.npy)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.combine:
        r64, r32 = (json.load(open(f)) for f in args.combine)
        res = compare(r64["cluster"], r64, r32)
    else:
        from synth.cluster import make_cluster
        from synth.workloads import MODEL_PP, WORKLOADS
        wl = WORKLOADS[args.workload]
        c = make_cluster(wl.radius_angstrom, wl.geometry_seed, wl.sigma)
        info = dict(workload=wl.name, n_si=c.n_si, n_h=c.n_h, n_atoms=c.n_atoms, degree=wl.degree)
        runs = {}
        for dt in ([args.only] if args.only else ["f64", "f32"]):
            runs[dt] = run_one(c, MODEL_PP, dt, wl.degree, log, args.sre_tol, args.max_steps, args.trace,
                               args.rho_in, args.rho_out)
            runs[dt]["cluster"] = info
            runs[dt]["start_density"] = os.path.basename(args.rho_in) if args.rho_in else "superposition"
        res = runs[args.only] if args.only else compare(info, runs["f64"], runs["f32"])
    log(json.dumps({k: v for k, v in res.items() if k not in ("eig_occ", "step_seconds")}))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()
