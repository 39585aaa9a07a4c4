#!/usr/bin/env python3
"""Single-GPU throughput of the Chebyshev filter Y = p_m(H) X.

One step = one chebyshev_filter call (degree m) over one block of vectors on
the full grid of the workload's cluster (inputs resident in HBM).  Metric:
filtered grid-point-vectors per second = N_points * n_vec / t_step.

Printed as one JSON line, with the roofline of the dominant kernel (the
Hilbert-tiled H X + recurrence kernel, timed with HIP events on its launch
stream inside the library) and the oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="d16nm")
    ap.add_argument("--dtype", default=None, choices=[None, "f32", "f64"])
    ap.add_argument("--nvec", type=int, default=None)
    ap.add_argument("--ordering", default="hilbert", choices=["hilbert", "lex"],
                    help="grid row order: blockwise Hilbert (tiled kernel) or lexicographic (neighbour-table kernel)")
    ap.add_argument("--generic", action="store_true",
                    help="use the neighbour-table kernel on the Hilbert order too (isolates the ordering effect)")
    ap.add_argument("--cpu-sample", default="auto",
                    help="oracle sample: 'auto' (0.55 nm grid x 1024 vectors) or 'workload:K' (this workload's "
                         "grid x K vectors)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--gram", type=int, default=0, metavar="M",
                    help="instead of the filter, time the Gram product X^T X of an M-column block over the "
                         "workload's rows (Cholesky-QR / Rayleigh-Ritz contraction) against the MFMA peak")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 4 GiB device copy (reference dispatch for HBM byte counters)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="JSON with counter-derived HBM bytes per H X launch for this workload")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 record (3 nm cluster, 128 FP64 vectors, degree 12: Hilbert-tiled kernel, "
                         "neighbour-table kernel on the Hilbert and on the lexicographic order)")
    return ap.parse_args()


def alg_bytes_per_launch(n_points: int, nvec: int, elem_bytes: int, degree: int) -> float:
    """Algorithmic HBM bytes of one H X + recurrence launch, averaged over a
    degree-m filter pass: every launch reads Y_k and writes Y_{k+1}, and all
    but the first also read Y_{k-1}, so a pass moves N nvec b (2 + 3 (m - 1))."""
    return n_points * nvec * elem_bytes * (2 + 3 * (degree - 1)) / degree


def kernel_source_hash() -> str:
    """SHA-256 of the H X kernel source without its // comments and blank
    lines (the counters in profiles/ name it; an edit of the comments alone
    leaves the kernels, and so the counters, unchanged)."""
    import hashlib
    src = os.path.join(ROOT, "paper_2303_00790_amd", "csrc", "hx.hip")
    with open(src, encoding="utf-8") as f:
        code = [line.split("//", 1)[0].rstrip() for line in f]
    return hashlib.sha256("\n".join(line for line in code if line).encode()).hexdigest()


def cpu_baseline(degree: int, sample: str = "auto", workload: str = "d16nm") -> dict:
    """The FP64 oracle filter timed on the host on a bounded sample: by
    default the 0.55 nm cluster's full grid (72,455 points) with 1024 vectors;
    'workload:K' takes the benched workload's own grid with K vectors."""
    import numpy as np
    from oracle import chfsi as OC
    from oracle import grid as OG
    from oracle import hamiltonian as OH
    from synth.cluster import make_cluster, random_block
    from synth.workloads import MODEL_PP, WORKLOADS
    if sample == "auto":
        wl, nvec = WORKLOADS["si35h36"], 1024
    else:
        kind, _, k = sample.partition(":")
        if kind != "workload" or not k.isdigit():
            raise SystemExit(f"bench.py: bad --cpu-sample {sample!r}")
        wl, nvec = WORKLOADS[workload], int(k)
    c = make_cluster(wl.radius_angstrom, wl.geometry_seed, wl.sigma)
    g = OG.build_grid(c.domain_radius(), wl.h)
    Ho = OH.build_hamiltonian(g, c.pos, c.species, OH.PseudoParams(**dataclasses.asdict(MODEL_PP)))
    X = random_block(g.n, nvec, wl.x_seed)
    b, tmin, _ = OC.lanczos_bound(Ho.apply, random_block(g.n, 1, wl.lanczos_seed)[:, 0])
    a0 = float(Ho.veff.min())
    a = tmin + 0.1 * (b - tmin)
    t0 = time.perf_counter()
    OC.chebyshev_filter(Ho.apply, X, degree, a, b, a0)
    dt = time.perf_counter() - t0
    return {"value": g.n * nvec / dt, "unit": "gridpt*vectors/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle degree-{degree} filter, {wl.name} grid ({g.n} points) x {nvec} vectors "
                      f"(scipy sparse stencil and projector products, single-threaded), {dt:.1f} s "
                      f"on {host_cpu()}"}


def host_cpu() -> str:
    """CPU model and visible logical CPUs of the host running the oracle."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return f"{model}, {n} logical CPUs visible"


MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}   # MI355X dense matrix peaks


def filter_record(B, H, X, W, degree, bounds, steps, warmup, generic, n_pts, nvec, es) -> dict:
    """Time `steps` degree-m filter calls (after `warmup`): throughput, the H X
    kernel's launches timed by the library, and both rooflines (the H X
    kernel per launch; the whole pass, every kernel included)."""
    import torch
    a, b, a0 = bounds
    for _ in range(warmup):
        H.filter(X, W, degree, a, b, a0, generic=generic)
    torch.cuda.synchronize()
    B.timer(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        H.filter(X, W, degree, a, b, a0, generic=generic)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tm = B.timer_read()
    B.timer(False)
    alg = alg_bytes_per_launch(n_pts, nvec, es, degree)
    hx_s = tm["hx_ms"] / 1e3 / max(1, tm["hx_launches"])
    pass_gbs = alg * degree / (ms / 1e3) / 1e9
    return {"ms_per_filter": ms, "value": n_pts * nvec / (ms / 1e3), "hx_avg_launch_ms": hx_s * 1e3,
            "kb_gather_avg_ms": tm["gather_ms"] / max(1, tm["gather_launches"]),
            "roofline": {"bound": "hbm", "achieved": alg / hx_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / hx_s / 1e9 / HBM_PEAK_GBS},
            "pass_achieved": pass_gbs, "pass_frac": pass_gbs / HBM_PEAK_GBS}


def committed_traffic(path: str, key: str):
    """HBM bytes per launch from the committed counter runs, only if they
    were taken on the kernel source as it is now (else None)."""
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(key)
    if rec and rec.get("source_sha256") == kernel_source_hash():
        return rec.get("bytes_per_launch")
    return None


def fp64_record(B, steps: int, warmup: int, traffic_path: str = "") -> dict:
    """The FP64 filter on the 3 nm cluster (Si705H300, 593,857 points): one
    128-vector block, degree 12, on the blockwise Hilbert order (tiled kernel,
    and the neighbour-table kernel on the same order) and on the
    lexicographic order (neighbour-table kernel)."""
    import torch
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP, WORKLOADS
    wl = WORKLOADS["d3nm"]
    c = make_cluster(wl.radius_angstrom, wl.geometry_seed, wl.sigma)
    radius = c.domain_radius()
    out = {"workload": f"{wl.name}: {wl.description}", "vectors": wl.nvec, "degree": wl.degree, "dtype": "f64"}
    ctx = B.Context(0)
    for name, ordering, generic in (("hilbert_tiled", B.ORDER_HILBERT, False),
                                    ("hilbert_neighbour_table", B.ORDER_HILBERT, True),
                                    ("lexicographic_neighbour_table", B.ORDER_LEX, True)):
        H = B.Hamiltonian(c.pos, c.species, MODEL_PP, wl.h, radius, ordering, keep_nbr=generic, dtypes=2)
        _, rows_np, _ = H.export_ordering()
        rows = torch.from_numpy(rows_np).cuda()
        inside = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
        inside[rows] = 1.0
        gen = torch.Generator(device="cuda")
        gen.manual_seed(wl.x_seed)
        X = torch.randn((H.n_rows, wl.nvec), generator=gen, dtype=torch.float64, device="cuda") * inside[:, None]
        W = torch.zeros_like(X)
        gen.manual_seed(wl.lanczos_seed)
        v0 = torch.randn(H.n_rows, generator=gen, dtype=torch.float64, device="cuda") * inside
        b, tmin, _ = H.lanczos_bound(ctx, v0, 10)
        a0 = float(H.vloc()[rows].min())
        out["points"] = H.n_points
        out[name] = filter_record(B, H, X, W, wl.degree, (tmin + 0.1 * (b - tmin), b, a0), steps, warmup, generic,
                                  H.n_points, wl.nvec, 8)
        if not generic:
            out[name]["roofline"]["traffic"] = committed_traffic(traffic_path, f"{wl.name}:f64:{wl.nvec}")
        del H, X, W
        torch.cuda.empty_cache()
    return out


def gram_bench(args, B, ctx, H, wl, dtype_name, tdtype, inside):
    """Time S = X^T X for an M-column block over all rows of the workload grid
    (the Gram product of Cholesky-QR and Rayleigh-Ritz): one JSON line with
    TFLOP/s counted as 2 N M^2 (the plain product; the library computes all of
    it) against the MFMA peak of the block dtype."""
    import torch
    m = args.gram
    gen = torch.Generator(device="cuda")
    gen.manual_seed(wl.x_seed)
    X = torch.randn((H.n_rows, m), generator=gen, dtype=tdtype, device="cuda")
    X.mul_(inside[:, None])
    S = torch.empty((m, m), dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        B.gram(ctx, X, X, S)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        B.gram(ctx, X, X, S)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flops = 2.0 * H.n_rows * m * m
    tf = flops / (ms / 1e3) / 1e12
    print(json.dumps({
        "metric": "Gram product X^T X TFLOP/s (2 N M^2 counted)", "value": tf, "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "rows": H.n_rows, "columns": m},
        "roofline": {"bound": "mfma", "achieved": tf, "peak": MFMA_PEAK_TFLOPS[dtype_name], "unit": "TFLOP/s",
                     "frac": tf / MFMA_PEAK_TFLOPS[dtype_name], "traffic": None}}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (--gpus {args.gpus} requested); "
              f"multi-GPU sharding is not provided", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2303_00790_amd import binding as B
    from synth.cluster import make_cluster
    from synth.workloads import MODEL_PP, WORKLOADS

    wl = WORKLOADS[args.workload]
    dtype_name = args.dtype or wl.dtype
    tdtype = torch.float32 if dtype_name == "f32" else torch.float64
    nvec = args.nvec or wl.nvec
    es = 4 if dtype_name == "f32" else 8
    torch.cuda.set_device(0)

    t_setup = time.perf_counter()
    c = make_cluster(wl.radius_angstrom, wl.geometry_seed, wl.sigma)
    radius = c.domain_radius()
    lex = args.ordering == "lex"
    H = B.Hamiltonian(c.pos, c.species, MODEL_PP, wl.h, radius, B.ORDER_LEX if lex else B.ORDER_HILBERT,
                      keep_nbr=lex or args.generic, dtypes=3)
    generic = lex or args.generic
    _, rows_np, _ = H.export_ordering()
    rows = torch.from_numpy(rows_np).cuda()
    inside = torch.zeros(H.n_rows, dtype=torch.bool, device="cuda")
    inside[rows] = True
    gen = torch.Generator(device="cuda")
    gen.manual_seed(wl.x_seed)
    X = torch.randn((H.n_rows, nvec), generator=gen, dtype=tdtype, device="cuda")
    X.mul_(inside[:, None])
    W = torch.zeros_like(X)
    gen.manual_seed(wl.lanczos_seed)
    v0 = torch.randn(H.n_rows, generator=gen, dtype=torch.float64, device="cuda") * inside
    ctx = B.Context(0)
    b, tmin, _ = H.lanczos_bound(ctx, v0, 10)
    vloc = H.vloc()
    a0 = float(vloc[inside].min())           # rigorous lower bound: -1/2 L >= 0, KB energies >= 0
    a = tmin + 0.1 * (b - tmin)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"# setup {t_setup:.1f} s: {H.n_points} points, {H.n_rows} rows, {H.n_blocks} blocks, "
          f"{H.n_proj} projector atoms, {H.n_pairs} pairs; bounds a0={a0:.4f} a={a:.4f} b={b:.4f}",
          file=sys.stderr, flush=True)
    if args.gram:
        gram_bench(args, B, ctx, H, wl, dtype_name, tdtype, inside)
        return

    for _ in range(args.warmup):
        H.filter(X, W, wl.degree, a, b, a0, generic=generic)
    torch.cuda.synchronize()
    B.timer(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        H.filter(X, W, wl.degree, a, b, a0, generic=generic)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    tm = B.timer_read()
    B.timer(False)
    if not bool(torch.isfinite(X).all()):
        print("bench.py: non-finite values in the filtered block", file=sys.stderr)
        sys.exit(3)

    n_pts = H.n_points
    value = n_pts * nvec / (ms / 1e3)
    launches = tm["hx_launches"]
    alg_bytes = alg_bytes_per_launch(n_pts, nvec, es, wl.degree)
    hx_avg_s = tm["hx_ms"] / 1e3 / max(1, launches)
    achieved = alg_bytes / hx_avg_s / 1e9
    # the whole pass (H X launches, KB gathers, everything between): the
    # algorithmic bytes of all degree steps over the measured time per pass
    pass_gbs = alg_bytes * wl.degree / (ms / 1e3) / 1e9
    # the staged tile kernel takes every block when no block has more than
    # 64 projector atoms (the case for all model clusters here; the trace in
    # the profile summaries names the kernel that ran)
    kernel = ("hx_generic_kernel" if generic else "hx_tile_kernel")
    # HBM traffic from the committed counter runs, only if they were taken on
    # the kernel source as it is now
    traffic = None if generic else committed_traffic(args.traffic, f"{wl.name}:{dtype_name}:{nvec}")
    out = {
        "metric": "filtered gridpt*vectors/s (Chebyshev filter, one GPU)",
        "value": value,
        "unit": "gridpt*vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "ordering": args.ordering, "kernel": kernel,
                   "points": n_pts, "rows": H.n_rows,
                   "vectors": nvec, "degree": wl.degree, "projector_atoms": H.n_proj, "h_bohr": wl.h,
                   "per_degree_rate": value * wl.degree},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "avg_launch_ms": hx_avg_s * 1e3,
                     "alg_bytes_per_launch": alg_bytes,
                     "kb_gather_avg_ms": tm["gather_ms"] / max(1, tm["gather_launches"]),
                     "kb_gather_launches": tm["gather_launches"],
                     "pass_achieved": pass_gbs, "pass_frac": pass_gbs / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    del X, W
    torch.cuda.empty_cache()
    if not args.no_fp64 and args.workload == "d16nm" and not generic:
        out["fp64_c2"] = fp64_record(B, max(3, args.steps // 2), 1, args.traffic)
    learned = os.path.join(ROOT, "results", "learned_density_4nm.json")
    if os.path.exists(learned):
        ld = json.load(open(learned))
        if "mean_steps_sad" in ld:
            out["scf_iters_saved"] = {"source": "results/learned_density_4nm.json (measured separately)",
                                      "clusters": len(ld.get("eval", [])), "dtype": ld.get("dtype"),
                                      "mean_steps_superposition": ld["mean_steps_sad"],
                                      "mean_steps_learned": ld["mean_steps_net"],
                                      "max_de_per_atom_ha": ld.get("max_de_per_atom")}
    if args.copy_calibration:
        src = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * 4
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl.degree, args.cpu_sample, wl.name)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
