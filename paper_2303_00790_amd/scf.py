"""SCF driver: runs scf_step through the C ABI until the SRE criterion holds.

Marshalling and the stop test only; every step of the method runs in the
library.  The paper's criterion is SRE < 1e-4 Ry with four ChFSI iterations
in the first SCF step and one in every later step.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class ScfResult:
    steps: int
    converged: bool
    energy: float
    eig: np.ndarray
    reports: list = field(default_factory=list)


def setup(cluster, pp, h: float = 0.7, dtype: str = "f64", degree: int = 10, nvec: int | None = None,
          x_seed: int = 2001, lanczos_seed: int = 3001, margin: float = 6.0, mix_beta: float = 0.1,
          mix_history: int = 8, first_iters: int = 4, work_cols: int = 256):
    """Hamiltonian, context, SCF state and the start block for a cluster.

    Anderson mixing defaults to beta = 0.1 with 8 past densities: at
    beta = 0.3 the density of clusters from 3 nm up sloshes without
    converging.  ``first_iters`` ChFSI iterations run in the first SCF step
    (the paper's schedule: 4, then 1 per step).  The work block has
    min(M, work_cols) columns: the filter and Rayleigh-Ritz run through it in
    column blocks and row panels, so X is the only block of full width (at
    5 nm in FP64, 151 GB for X against 5 GB of work)."""
    import torch
    from synth.cluster import n_states
    radius = cluster.domain_radius(margin)
    H = B.Hamiltonian(cluster.pos, cluster.species, pp, h, radius, B.ORDER_HILBERT, dtypes=3)
    ctx = B.Context(0)
    ne = cluster.n_electrons
    M = nvec or n_states(ne)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    code = B.CHF_F64 if dtype == "f64" else B.CHF_F32
    _, rows_np, _ = H.export_ordering()
    rows = torch.from_numpy(rows_np).cuda()
    # start block: i.i.d. N(0, 1) drawn in FP64 on the device (seeded; the
    # same numbers for either work dtype), written to the inside rows in
    # row chunks so no FP64 copy of the whole block is needed
    gen = torch.Generator(device="cuda")
    gen.manual_seed(x_seed)
    X = torch.zeros((H.n_rows, M), dtype=tdt, device="cuda")
    step = max(1, (1 << 27) // M)
    for r0 in range(0, H.n_points, step):
        r = rows[r0:r0 + step]
        X[r] = torch.randn((r.numel(), M), generator=gen, dtype=torch.float64, device="cuda").to(tdt)
    v0 = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
    v0[rows] = torch.from_numpy(np.random.default_rng(lanczos_seed).standard_normal(H.n_points)).cuda()
    eii = B.ion_energy(cluster.pos, cluster.species, pp)
    prm = B.ScfParams(ne, M, degree, first_iters, 1, 10, code, code, mix_history, mix_beta, 1e-12, eii)
    W = torch.zeros((H.n_rows, min(M, work_cols)), dtype=tdt, device="cuda")
    return dict(H=H, ctx=ctx, prm=prm, X=X, W=W, v0=v0, rows=rows, ne=ne, M=M)


def run(state, rho0, max_steps: int = 60, sre_tol_ry: float = 1e-4, min_steps: int = 1, log=None,
        trace=None) -> ScfResult:
    """SCF steps until SRE < sre_tol_ry; ``log`` (optional) receives one
    line per step; ``trace`` (optional path or writable text file) receives
    one JSON object per step: the step report (SRE, energies, HOMO/LUMO,
    filter bounds, ChFSI and CG iterations, Cholesky-QR fallbacks) and the
    step's wall time in seconds."""
    import json
    import time
    import torch
    scf = B.Scf(state["H"], state["ctx"], state["prm"], rho0, state["v0"])
    reps = []
    eig = None
    converged = False
    own = isinstance(trace, (str, bytes, os.PathLike))
    tf = open(trace, "a") if own else trace
    try:
        for _ in range(max_steps):
            t0 = time.perf_counter()
            rep, eig = scf.step(state["X"], state["W"])
            torch.cuda.synchronize()
            d = rep.as_dict()
            d["seconds"] = time.perf_counter() - t0
            reps.append(d)
            if tf is not None:
                tf.write(json.dumps(d) + "\n")
                tf.flush()
            if log is not None:
                log(f"  scf step {rep.step}: SRE {rep.sre_ry:.3e} Ry, E {rep.energy:.8f} Ha")
            if rep.sre_ry < sre_tol_ry and rep.step >= min_steps:
                converged = True
                break
    finally:
        if own:
            tf.close()
    state["scf"] = scf
    return ScfResult(len(reps), converged, reps[-1]["energy"], eig, reps)
