"""Shared GPU test inputs: the 0.55 nm Si35H36 cluster (seed 1001) on its
h = 0.7 bohr sphere, with matching oracle and device Hamiltonians."""
import numpy as np

from oracle import grid as G
from oracle import hamiltonian as OH
from synth.cluster import make_cluster


def build(pp=None, veff_seed=77, ordering=G.ORDER_HILBERT, h=0.7, radius_angstrom=5.5, keep_nbr=True):
    import torch
    from paper_2303_00790_amd import binding as B
    c = make_cluster(radius_angstrom, 1001)
    radius = c.domain_radius()
    pp = pp or OH.PseudoParams(h_s=2.0, h_p=0.5)
    g = G.build_grid(radius, h, ordering)
    Ho = OH.build_hamiltonian(g, c.pos, c.species, pp)
    if veff_seed is not None:
        rng = np.random.default_rng(veff_seed)
        Ho.veff = Ho.vloc + 0.05 * np.sin(g.xyz @ rng.standard_normal(3))
    Hg = B.Hamiltonian(c.pos, c.species, pp, h, radius, ordering, keep_nbr=keep_nbr)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    veff_rows = torch.zeros(Hg.n_rows, dtype=torch.float64, device="cuda")
    veff_rows[rows] = torch.from_numpy(Ho.veff).cuda()
    Hg.set_veff(veff_rows)
    return dict(B=B, c=c, g=g, Ho=Ho, Hg=Hg, rows=rows, pp=pp, radius=radius)


def to_rows(s, X, dtype, ld=None):
    import torch
    X = np.asarray(X)
    if X.ndim == 1:
        out = torch.zeros(s["Hg"].n_rows, dtype=dtype, device="cuda")
        out[s["rows"]] = torch.from_numpy(X).to(device="cuda", dtype=dtype)
        return out
    n, m = X.shape
    ld = ld or m
    out = torch.zeros((s["Hg"].n_rows, ld), dtype=dtype, device="cuda")
    out[s["rows"], :m] = torch.from_numpy(X).to(device="cuda", dtype=dtype)
    return out


def from_rows(s, Y, m=None):
    if Y.dim() == 1:
        return Y[s["rows"]].double().cpu().numpy()
    return Y[s["rows"], :m].double().cpu().numpy()


def relerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())
