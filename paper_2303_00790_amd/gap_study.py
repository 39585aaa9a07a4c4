"""Size dependence of the gap and the density of states on model clusters,
and the grid-spacing check (Results section: DOS with 0.1 eV bins aligned at
the highest occupied state; gap(d) = E0 + A / d^k; spectra at h = 0.9 bohr
against h = 0.7 bohr).

    python -m paper_2303_00790_amd.gap_study --diam 1.0 1.5 2.0 2.5 3.0 --h2 0.9 --out gap.json
    python -m paper_2303_00790_amd.gap_study --diam 5.0 --seed0 30007 --h2 0.9 --out gap5.json
    python -m paper_2303_00790_amd.gap_study --merge gap.json gap5.json --out gap_all.json
    python -m paper_2303_00790_amd.gap_study --diam 5.0 --seed0 30007 --h2 0.9 --rho-in rho5.npy --out gap5.json

Each cluster (seed seed0 + i, position noise 0.02 angstrom) is converged by
the library's SCF to SRE < 1e-4 Ry in the mixed-precision mode; the
eigenvalues, HOMO-LUMO gap and DOS (0.1 eV bins, HOMO at 0) are recorded, the
gap is fitted, and with --h2 every cluster is converged again at the second
spacing and the two spectra compared.  --merge joins the cluster lists of
several runs (same spacing, precision and pseudopotential) and refits.
--rho-in starts the first cluster's SCF at spacing --h from a stored density
(a pre-converged one, to split a long SCF); the second spacing starts from
the superposition.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def converge(cluster, pp, h: float, dtype: str, degree: int, log, rho_in=None):
    """The SCF of one cluster at spacing h from the superposition start, or
    from rho_in (.npy of the inside-point values in curve order, made on the
    same grid)."""
    import torch
    from . import scf as S
    st = S.setup(cluster, pp, h=h, dtype=dtype, degree=degree)
    H = st["H"]
    if rho_in:
        rho = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
        vals = torch.from_numpy(np.load(rho_in)).cuda()
        if vals.numel() != st["rows"].numel():
            raise SystemExit(f"gap_study: {rho_in} holds {vals.numel()} points, the grid {st['rows'].numel()}")
        rho[st["rows"]] = vals
    else:
        rho = H.sad_density(cluster.pos, cluster.species, cluster.n_electrons)
    t0 = time.perf_counter()
    log(f"cluster Si{cluster.n_si}H{cluster.n_h}, h = {h}: {H.n_points} points, {st['M']} states")
    res = S.run(st, rho, max_steps=80, sre_tol_ry=1e-4, log=log)
    dt = time.perf_counter() - t0
    out = dict(n_points=H.n_points, M=st["M"], n_occ=cluster.n_electrons // 2, steps=res.steps,
               converged=res.converged, energy=res.energy, eig=np.asarray(res.eig, dtype=np.float64), seconds=dt)
    del st, H
    torch.cuda.empty_cache()
    return out


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from . import analysis as A
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--diam", type=float, nargs="+", default=[1.0, 1.5, 2.0, 2.5, 3.0])
    ap.add_argument("--h", type=float, default=0.7)
    ap.add_argument("--h2", type=float, default=None)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--degree", type=int, default=12)
    ap.add_argument("--pp", default="", help="model pseudopotential overrides, e.g. r_loc=0.9,h_s=2.0")
    ap.add_argument("--seed0", type=int, default=30000, help="geometry seed of the first diameter")
    ap.add_argument("--merge", nargs="+", default=None, metavar="JSON", help="join earlier runs and refit")
    ap.add_argument("--rho-in", default=None,
                    help="start density of the first cluster at spacing --h (.npy, inside points in curve order)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    pp = MODEL_PP
    if args.pp:
        import dataclasses
        pp = dataclasses.replace(MODEL_PP, **{k: float(v) for k, v in (kv.split("=") for kv in args.pp.split(","))})

    def log(msg):
        print(msg, flush=True)

    if args.merge:
        runs = [json.load(open(f)) for f in args.merge]
        for key in ("h", "dtype", "pp"):
            if any(r.get(key) != runs[0].get(key) for r in runs):
                raise SystemExit(f"gap_study --merge: the runs differ in {key}")
        rows = sorted((c for r in runs for c in r["clusters"]), key=lambda c: c["diam_nm"])
        res = dict(h=runs[0]["h"], dtype=runs[0]["dtype"], pp=runs[0]["pp"], clusters=rows,
                   merged_from=[os.path.basename(f) for f in args.merge])
        fit_and_write(res, rows, args.out, log)
        return res
    rows = []
    for i, d in enumerate(args.diam):
        c = make_cluster(5.0 * d, args.seed0 + i, sigma_angstrom=0.02)
        start = args.rho_in if i == 0 else None
        r = converge(c, pp, args.h, args.dtype, args.degree, log, rho_in=start)
        row = dict(diam_nm=d, seed=args.seed0 + i, start_density=os.path.basename(start) if start else "superposition", n_si=c.n_si, n_h=c.n_h, n_points=r["n_points"], states=r["M"],
                   n_occ=r["n_occ"],
                   steps=r["steps"], converged=r["converged"], energy=r["energy"], seconds=r["seconds"],
                   gap_ev=A.gap_ev(r["eig"], r["n_occ"]))
        centres, dens = A.dos_histogram(r["eig"], r["n_occ"])
        row.update(dos_bin_centres_ev=[float(x) for x in centres], dos=[float(x) for x in dens])
        if args.h2:
            r2 = converge(c, pp, args.h2, args.dtype, args.degree, log)
            _, dens2 = A.dos_histogram(r2["eig"], r2["n_occ"])
            row["dos_h2"] = [float(x) for x in dens2]
            occ = slice(0, r["n_occ"])
            e1 = (r["eig"][occ] - r["eig"][r["n_occ"] - 1]) * A.HARTREE_EV
            e2 = (r2["eig"][occ] - r2["eig"][r["n_occ"] - 1]) * A.HARTREE_EV
            row.update(h2=args.h2, n_points_h2=r2["n_points"], gap_ev_h2=A.gap_ev(r2["eig"], r2["n_occ"]),
                       steps_h2=r2["steps"], dos_rms_h_vs_h2=A.dos_rms(dens, dens2),
                       occ_shift_mean_abs_ev=float(np.mean(np.abs(e1 - e2))),
                       occ_shift_max_abs_ev=float(np.max(np.abs(e1 - e2))))
        log(json.dumps(row))
        rows.append(row)
    import dataclasses
    res = dict(h=args.h, dtype=args.dtype, pp=dataclasses.asdict(pp), clusters=rows)
    fit_and_write(res, rows, args.out, log)
    return res


def fit_and_write(res: dict, rows: list, out, log) -> None:
    from . import analysis as A
    if len(rows) >= 3:
        dd, gg = [r["diam_nm"] for r in rows], [r["gap_ev"] for r in rows]
        e0, a, k, r2 = A.fit_gap(dd, gg)
        res["fit"] = dict(e0_ev=e0, a_ev=a, k=k, r2=r2)
        log(f"gap fit: E0 = {e0:.3f} eV, A = {a:.3f} eV, k = {k:.3f}, R^2 = {r2:.5f}")
        e0, a, k, r2 = A.fit_gap(dd, gg, k=1.56)
        res["fit_k_1.56"] = dict(e0_ev=e0, a_ev=a, k=k, r2=r2)
        log(f"gap fit at the published exponent 1.56: E0 = {e0:.3f} eV, A = {a:.3f} eV, R^2 = {r2:.5f}")
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
