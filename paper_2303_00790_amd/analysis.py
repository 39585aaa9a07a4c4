"""Electronic-structure post-processing of converged SCF runs: density of
states and the size dependence of the HOMO-LUMO gap (Results section: DOS
histograms with 0.1 eV bins aligned at the highest occupied state, areas
normalised below it; gap fitted to E0 + A / d^k with d in nm).

Host-side NumPy on a few thousand eigenvalues; nothing here is on the hot
path.
"""
from __future__ import annotations

import math

import numpy as np

HARTREE_EV = 27.211386245988


def dos_histogram(eig_ha, n_occ: int, bin_ev: float = 0.1, lo_ev: float = -15.0, hi_ev: float = 5.0,
                  area: float = 1.0):
    """DOS of one cluster.

    Eigenvalues are shifted so that the highest occupied state (index
    n_occ - 1 of the ascending list) sits at 0 eV and binned on edges
    k * bin_ev; a value on an edge belongs to the bin below it, so the
    highest occupied state falls in (-bin_ev, 0].  The counts are scaled so
    that the area (sum of count * bin width) below 0 eV equals ``area``.

    Returns (edges_ev, density): len(edges) = len(density) + 1.
    """
    e = np.sort(np.asarray(eig_ha, dtype=np.float64)) * HARTREE_EV
    if not 0 < n_occ <= e.size:
        raise ValueError("n_occ must be in [1, number of eigenvalues]")
    e = e - e[n_occ - 1]
    k_lo = math.floor(lo_ev / bin_ev + 1e-9)
    k_hi = math.ceil(hi_ev / bin_ev - 1e-9)
    edges = np.arange(k_lo, k_hi + 1) * bin_ev
    # bin index: smallest k with e <= edges[k], minus one  (right-closed bins)
    idx = np.searchsorted(edges, e, side="left") - 1
    keep = (idx >= 0) & (idx < edges.size - 1)
    counts = np.bincount(idx[keep], minlength=edges.size - 1).astype(np.float64)
    below = counts[edges[1:] <= 1e-12].sum() * bin_ev
    density = counts * (area / below) if below > 0 else counts
    return edges, density


def dos_rms(d1, d2) -> float:
    """RMS difference of two DOS curves sampled on the same bins."""
    d1 = np.asarray(d1, dtype=np.float64)
    d2 = np.asarray(d2, dtype=np.float64)
    if d1.shape != d2.shape:
        raise ValueError("DOS curves must share their bins")
    return float(np.sqrt(np.mean((d1 - d2) ** 2)))


def gap_ev(eig_ha, n_occ: int) -> float:
    """HOMO-LUMO gap in eV from an ascending (or unsorted) eigenvalue list."""
    e = np.sort(np.asarray(eig_ha, dtype=np.float64))
    if not 0 < n_occ < e.size:
        raise ValueError("need at least one empty state above the n_occ occupied ones")
    return float((e[n_occ] - e[n_occ - 1]) * HARTREE_EV)


def fit_gap(d_nm, gap, p0=(0.5, 4.0, 1.5), k: float | None = None):
    """Least-squares fit of gap(d) = E0 + A / d^k; returns (E0, A, k, R^2).
    With ``k`` given only E0 and A are fitted (a linear least-squares
    problem in 1 / d^k)."""
    d = np.asarray(d_nm, dtype=np.float64)
    g = np.asarray(gap, dtype=np.float64)
    if k is not None:
        if d.size < 2:
            raise ValueError("need at least two sizes for a two-parameter fit")
        A_mat = np.stack([np.ones_like(d), d ** -float(k)], axis=1)
        (e0, a), *_ = np.linalg.lstsq(A_mat, g, rcond=None)
        res = g - A_mat @ np.array([e0, a])
        ss_tot = float(((g - g.mean()) ** 2).sum())
        r2 = 1.0 - float((res ** 2).sum()) / ss_tot if ss_tot > 0 else 1.0
        return float(e0), float(a), float(k), r2
    from scipy.optimize import curve_fit
    if d.size < 3:
        raise ValueError("need at least three sizes for a three-parameter fit")

    def model(x, e0, a, k):
        return e0 + a / x ** k

    p, _ = curve_fit(model, d, g, p0=p0, maxfev=20000)
    res = g - model(d, *p)
    ss_tot = float(((g - g.mean()) ** 2).sum())
    r2 = 1.0 - float((res ** 2).sum()) / ss_tot if ss_tot > 0 else 1.0
    return float(p[0]), float(p[1]), float(p[2]), r2
