"""Learned initial SCF density: data generation, training and evaluation.

The network (dnet_* in the library) maps the scaled superposition-of-atoms
density on a cubic patch of the grid to a scaled correction towards the
converged SCF density.  Training data are converged densities that the
method itself produces on seeded random clusters; evaluation compares the
number of SCF steps to reach the paper's criterion (SRE < 1e-4 Ry) from the
plain superposition start and from the corrected start, at equal converged
energy.  This module only marshals data and drives the loop; every
numerical step runs in the library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from . import scf as S

SCALE = 30.0        # densities (e/bohr^3, ~0.03 in bulk Si) scaled to O(1)


@dataclass
class Sample:
    box_sad: object      # torch float32 [D^3], scaled SAD density
    box_delta: object    # torch float32 [D^3], scaled (rho_conv - rho_sad)
    D: int
    n_atoms: int
    steps: int


def box_geometry(H) -> tuple[int, int]:
    """Edge D (multiple of 8) and offset of the grid origin in the box."""
    ijk, _, _ = H.export_ordering()
    n_r = int(np.abs(ijk).max())
    D = ((2 * n_r + 1 + 7) // 8) * 8
    return D, n_r + (D - (2 * n_r + 1)) // 2


def converged_sample(cluster, pp, dtype: str = "f32", sre_tol_ry: float = 1e-4, max_steps: int = 60, log=None,
                     start_net=None, start_highpass: float = 0.0):
    """One training sample: the SCF converged from the superposition start,
    or from start_net's predicted start (the fixed point, and so the label,
    is the same; only the number of steps to reach it changes)."""
    import torch
    st = S.setup(cluster, pp, dtype=dtype)
    H = st["H"]
    if start_net is not None:
        rho_sad, rho0 = predicted_start(start_net, H, cluster, start_highpass)
    else:
        rho_sad = H.sad_density(cluster.pos, cluster.species, cluster.n_electrons)
        rho0 = rho_sad.clone()
    res = S.run(st, rho0, max_steps=max_steps, sre_tol_ry=sre_tol_ry, log=log)
    rho_conv = torch.zeros_like(rho_sad)
    st["scf"].fields(rho_conv)
    D, off = box_geometry(H)
    bs = torch.zeros(D ** 3, dtype=torch.float32, device="cuda")
    bd = torch.zeros_like(bs)
    B.rows_to_box(H, rho_sad, SCALE, bs, D, off)
    B.rows_to_box(H, rho_conv, SCALE, bd, D, off, base=rho_sad)      # the label: rho_conv - rho_sad
    return Sample(bs, bd, D, cluster.n_atoms, res.steps), res


def make_dataset(n: int, seed0: int, diam_nm: tuple[float, float], pp, sigma: float = 0.05, log=print,
                 dtype: str = "f64", budget_s: float | None = None, start_net=None, start_highpass: float = 0.0):
    """Training data: the superposition start and the correction to the SCF
    density converged by the FP64 path (dtype) on up to n seeded random
    clusters; with budget_s, no new cluster is started once that many seconds
    have passed (the data stay in device memory, so generation and training
    share one session).  start_net (an earlier network) only shortens the
    SCFs that make the labels."""
    from synth.cluster import make_cluster
    rng = np.random.default_rng(seed0)
    data = []
    t_start = time.perf_counter()
    for i in range(n):
        if budget_s is not None and time.perf_counter() - t_start > budget_s:
            log(f"data budget of {budget_s:.0f} s reached after {len(data)} clusters")
            break
        d = float(rng.uniform(*diam_nm))
        c = make_cluster(5.0 * d, seed0 + i, sigma_angstrom=sigma)
        if c.n_atoms == 0:
            continue
        t0 = time.perf_counter()
        smp, res = converged_sample(c, pp, dtype=dtype, log=log, start_net=start_net,
                                    start_highpass=start_highpass)
        data.append(smp)
        log(f"train cluster {i}: d={d:.2f} nm Si{c.n_si}H{c.n_h} box {smp.D}^3 scf steps {res.steps} "
            f"converged {res.converged} ({time.perf_counter() - t0:.1f} s)")
    return data


def train(net, data, steps: int, patch: int = 64, lr: float = 1e-3, seed: int = 0, log=print):
    import torch
    rng = np.random.default_rng(seed)
    x = torch.zeros(patch ** 3, dtype=torch.float32, device="cuda")
    t = torch.zeros_like(x)
    y = torch.zeros_like(x)
    dy = torch.zeros_like(x)
    losses = []
    for step in range(1, steps + 1):
        smp = data[int(rng.integers(len(data)))]
        lo = -patch // 4
        hi = max(lo + 1, smp.D - 3 * patch // 4)
        o = rng.integers(lo, hi, size=3)
        sym = int(rng.integers(48))
        B.crop(smp.box_sad, smp.D, patch, o, sym, x)
        B.crop(smp.box_delta, smp.D, patch, o, sym, t)
        net.forward(x, y)
        losses.append(net.mse(y, t, dy))
        net.backward(dy)
        net.adam(lr, step)
        if step % max(1, steps // 10) == 0:
            log(f"train step {step}: loss {np.mean(losses[-max(1, steps // 10):]):.3e}")
    return losses


def predicted_start(net, H, cluster, highpass_sigma: float = 0.0):
    """rho_0 = renormalise(max(rho_sad + net(rho_sad), 0)) on the full box.

    With highpass_sigma > 0 (cells) only the part of the predicted correction
    above the Gaussian's wavelengths is kept: the network reproduces the
    bond-scale correction but misses its long-wavelength charge shifts, which
    the Hartree potential amplifies."""
    import torch
    rho_sad = H.sad_density(cluster.pos, cluster.species, cluster.n_electrons)
    D, off = box_geometry(H)
    box = torch.zeros(D ** 3, dtype=torch.float32, device="cuda")
    B.rows_to_box(H, rho_sad, SCALE, box, D, off)
    out = torch.zeros_like(box)
    net.forward(box, out)
    if highpass_sigma > 0:
        work = torch.zeros(2 * D ** 3, dtype=torch.float32, device="cuda")
        hp = torch.zeros_like(box)
        B.highpass(out, D, highpass_sigma, hp, work)
        out = hp
        del work
    rho0 = torch.zeros_like(rho_sad)
    B.box_to_rows(H, out, D, off, SCALE, rho_sad, rho0)
    H.density_fix(rho0, cluster.n_electrons)
    return rho_sad, rho0


def evaluate(net, clusters, pp, dtype: str = "f64", sre_tol_ry: float = 1e-4, log=print, first_iters: int = 4,
             highpass_sigma: float = 0.0):
    """SCF from the superposition start and from the learned start, same
    schedule and start vectors; steps to SRE < sre_tol_ry and energies."""
    rows = []
    for c in clusters:
        st = S.setup(c, pp, dtype=dtype, first_iters=first_iters)
        rho_sad, rho0 = predicted_start(net, st["H"], c, highpass_sigma)
        log(f"eval Si{c.n_si}H{c.n_h}: from the superposition start")
        r_sad = S.run(st, rho_sad, max_steps=80, sre_tol_ry=sre_tol_ry, log=log)
        st2 = S.setup(c, pp, dtype=dtype, first_iters=first_iters)
        _, rho0b = predicted_start(net, st2["H"], c, highpass_sigma)
        log(f"eval Si{c.n_si}H{c.n_h}: from the learned start")
        r_net = S.run(st2, rho0b, max_steps=80, sre_tol_ry=sre_tol_ry, log=log)
        row = dict(n_atoms=c.n_atoms, steps_sad=r_sad.steps, steps_net=r_net.steps, conv_sad=r_sad.converged,
                   conv_net=r_net.converged, e_sad=r_sad.energy, e_net=r_net.energy,
                   de_per_atom=abs(r_sad.energy - r_net.energy) / c.n_atoms,
                   sre0_sad=r_sad.reports[0]["sre_ry"], sre0_net=r_net.reports[0]["sre_ry"])
        log(f"eval Si{c.n_si}H{c.n_h}: steps SAD {r_sad.steps} vs learned {r_net.steps}, "
            f"|dE|/atom {row['de_per_atom']:.2e} Ha, first SRE {row['sre0_sad']:.3e} vs {row['sre0_net']:.3e}")
        rows.append(row)
        del st, st2
    return rows
