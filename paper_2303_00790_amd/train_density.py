"""Train the initial-density network on converged densities and evaluate the
SCF steps it saves.

    python -m paper_2303_00790_amd.train_density --train 40 --steps 1500 --eval 3 --out results.json

Training clusters: seeded random H-passivated Si spheres (diameters drawn
uniformly from --train-diam, position noise 0.05 angstrom), each converged
with the SCF to SRE < 1e-4 Ry.  Evaluation clusters use unseen seeds and
--eval-diam; each runs the SCF from the superposition start and from the
network's start, reporting steps to convergence and the energy difference.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def main(argv=None):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from paper_2303_00790_amd import binding as B
    from paper_2303_00790_amd import density_model as DM
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP

    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--train-diam", type=float, nargs=2, default=(1.5, 3.0))
    ap.add_argument("--data-budget", type=float, default=None, metavar="SECONDS",
                    help="stop generating training clusters after this many seconds")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--patch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--eval", type=int, default=3)
    ap.add_argument("--eval-diam", type=float, default=3.0)
    ap.add_argument("--dtype", default="f64", help="SCF precision of the training labels and the evaluation")
    ap.add_argument("--eval-seed", type=int, default=20000)
    ap.add_argument("--first-iters", type=int, default=4, help="ChFSI iterations in the first SCF step of the evaluation")
    ap.add_argument("--highpass", type=float, default=0.0,
                    help="keep only the correction above this Gaussian width (grid cells); 0 keeps all of it")
    ap.add_argument("--out", default=None)
    ap.add_argument("--params-out", default=None)
    ap.add_argument("--params-in", default=None, help="skip data and training; evaluate these weights")
    ap.add_argument("--label-start", default=None, metavar="NPY",
                    help="weights of an earlier network whose (high-passed) prediction starts the SCFs that make "
                         "the training labels; the labels are the same converged densities, reached in fewer steps")
    ap.add_argument("--merge", nargs="+", default=None, metavar="JSON",
                    help="combine a training record and evaluation records (same weights, same diameter) into --out")
    ap.add_argument("--test-record", default=None, metavar="JSON",
                    help="with --merge: an evaluation record of one small cluster, kept as the test case")
    args = ap.parse_args(argv)
    if args.merge:
        res = merge_records(args.merge, args.test_record)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(res, f, indent=1)
        print(json.dumps({k: v for k, v in res.items() if k != "eval"}))
        return

    def log(msg):
        print(msg, flush=True)

    net = B.DensityNet(args.channels, seed=1)
    res = {"channels": args.channels, "dtype": args.dtype}
    if args.params_in:
        net.set_params(np.load(args.params_in).astype(np.float32))
        res["params_in"] = os.path.basename(args.params_in)
    else:
        t0 = time.perf_counter()
        start_net = None
        if args.label_start:
            start_net = B.DensityNet(args.channels, seed=2)
            start_net.set_params(np.load(args.label_start).astype(np.float32))
            res["label_start"] = {"params": os.path.basename(args.label_start), "highpass_sigma": args.highpass}
        data = DM.make_dataset(args.train, 10000, tuple(args.train_diam), MODEL_PP, sigma=0.05, log=log,
                               dtype=args.dtype, budget_s=args.data_budget, start_net=start_net,
                               start_highpass=args.highpass)
        del start_net
        t_data = time.perf_counter() - t0
        t1 = time.perf_counter()
        losses = DM.train(net, data, args.steps, patch=args.patch, lr=args.lr, log=log)
        t_train = time.perf_counter() - t1
        res.update({"train_clusters": len(data), "train_clusters_requested": args.train, "dtype": args.dtype,
                    "train_diam_nm": list(args.train_diam), "steps": args.steps,
                    "patch": args.patch, "data_s": t_data, "train_s": t_train,
                    "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(losses[-20:]))})
        if args.params_out:
            np.save(args.params_out, net.get_params())
        del data
    if args.eval > 0:
        evals = [make_cluster(5.0 * args.eval_diam, args.eval_seed + i, sigma_angstrom=0.02) for i in range(args.eval)]
        rows = DM.evaluate(net, evals, MODEL_PP, dtype=args.dtype, log=log, first_iters=args.first_iters,
                           highpass_sigma=args.highpass)
        res.update({"eval_diam_nm": args.eval_diam, "eval_seeds": [args.eval_seed + i for i in range(args.eval)],
                    "first_iters": args.first_iters, "highpass_sigma": args.highpass,
                    "eval": rows, "mean_steps_sad": float(np.mean([r["steps_sad"] for r in rows])),
                    "mean_steps_net": float(np.mean([r["steps_net"] for r in rows])),
                    "max_de_per_atom": float(max(r["de_per_atom"] for r in rows))})
    log(json.dumps(res))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)


def merge_records(paths, test_path=None) -> dict:
    """One record from a training run and evaluation runs of its weights:
    the training fields, the evaluation rows of all runs in order, their
    means, and (test_path) one small cluster's evaluation as the test case."""
    recs = [json.load(open(p)) for p in paths]
    train = next((r for r in recs if "train_clusters" in r), None)
    evals = [r for r in recs if r.get("eval")]
    diams = {r["eval_diam_nm"] for r in evals}
    sigmas = {r["highpass_sigma"] for r in evals}
    dtypes = {r["dtype"] for r in evals}
    if len(diams) > 1 or len(sigmas) > 1 or len(dtypes) > 1:
        raise SystemExit("merge: evaluation records differ in diameter, high-pass width or dtype")
    rows = [row for r in evals for row in r["eval"]]
    res = {"channels": (train or evals[0])["channels"], "dtype": dtypes.pop() if dtypes else None,
           "train": {k: v for k, v in (train or {}).items() if k not in ("eval",)},
           "eval_diam_nm": diams.pop() if diams else None,
           "eval_seeds": [s for r in evals for s in r["eval_seeds"]],
           "first_iters": evals[0]["first_iters"] if evals else None,
           "highpass_sigma": sigmas.pop() if sigmas else None,
           "eval": rows}
    if rows:
        res.update({"mean_steps_sad": float(np.mean([r["steps_sad"] for r in rows])),
                    "mean_steps_net": float(np.mean([r["steps_net"] for r in rows])),
                    "max_de_per_atom": float(max(r["de_per_atom"] for r in rows))})
    if test_path:
        # the first cluster of that record is the test case; all its rows are kept
        t = json.load(open(test_path))
        row = t["eval"][0]
        res["test_cluster"] = {"diam_nm": t["eval_diam_nm"], "seed": t["eval_seeds"][0],
                               "highpass_sigma": t["highpass_sigma"], "dtype": t["dtype"],
                               "steps_sad": row["steps_sad"], "steps_net": row["steps_net"],
                               "de_per_atom": row["de_per_atom"]}
        res["small_clusters"] = {"diam_nm": t["eval_diam_nm"], "seeds": t["eval_seeds"], "eval": t["eval"]}
    return res


if __name__ == "__main__":
    main()
