"""Named synthetic workloads (inputs and run sizes) and the model constants.

The five workloads follow the paper's system class -- spherical, H-passivated
Si nanoclusters cut from the diamond lattice on an h = 0.7 bohr grid -- at
sizes one GPU holds: a 0.55 nm-radius cluster for full SCF parity, 3 nm and
5 nm clusters for the FP64 and mixed-precision paths, 4 nm clusters for the
learned initial density, and a 16 nm cluster (the diameter of the paper's
largest nanocluster, Si107641H9084 in Table I) for the single-GPU filter
throughput.  Seeds: geometry 1000 + k, vectors 2000 + k, Lanczos start
3000 + k for workload k.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class ModelPP:
    """Model pseudopotential constants (the paper's Troullier-Martins tables
    are not available; an analytic erf local part and Gaussian s/p KB
    projectors on Si stand in)."""
    z_si: float = 4.0
    z_h: float = 1.0
    r_loc: float = 0.7       # erf width of the Si local part (bohr)
    r_loc_h: float = 0.5     # erf width of the H local part (bohr)
    r_c: float = 1.2         # Gaussian projector width (bohr)
    r_cut: float = 4.8       # projector cutoff (bohr)
    h_s: float = 3.0         # KB energy, s channel (Ha)
    h_p: float = 0.0         # KB energy, p channel (Ha)


MODEL_PP = ModelPP()


@dataclass(frozen=True)
class Workload:
    name: str
    description: str
    radius_angstrom: float     # cluster cut radius
    k: int                     # workload index (seeds 1000 + k, 2000 + k, 3000 + k)
    h: float = 0.7             # grid spacing, bohr
    degree: int = 10
    nvec: int = 128            # vectors filtered per call
    dtype: str = "f64"
    sigma: float = 0.02        # position noise, angstrom

    @property
    def geometry_seed(self) -> int:
        return 1000 + self.k

    @property
    def x_seed(self) -> int:
        return 2000 + self.k

    @property
    def lanczos_seed(self) -> int:
        return 3000 + self.k


WORKLOADS = {
    "si35h36": Workload("si35h36", "0.55 nm-radius Si35H36, FP64 ChFSI SCF", 5.5, 1, degree=10, nvec=128),
    "d3nm": Workload("d3nm", "3 nm Si705H300, FP64 filter on 128-vector blocks", 15.0, 2, degree=12, nvec=128),
    "d5nm": Workload("d5nm", "5 nm Si3205H828, mixed precision", 25.0, 3, degree=12, nvec=256, dtype="f32"),
    "d4nm": Workload("d4nm", "4 nm Si1683H580, learned-density evaluation", 20.0, 4, degree=12, nvec=4032),
    "d16nm": Workload("d16nm", "16 nm Si107041H9060, one degree-16 FP32 filter pass on 256 vectors", 80.0, 5,
                      degree=16, nvec=256, dtype="f32"),
}


# Constants of the method shared by every workload (the readings of the
# paper's silent points; the defaults the drivers use).
METHOD = {
    "fd_half_order": 6,                 # 12th-order central second derivative, 37-point star
    "block_edge": 8,                    # Hilbert blocks of 8^3 points
    "domain_margin_bohr": 6.0,          # R_domain = max |r_atom| + margin
    "lanczos_steps": 10,
    "chfsi_iters_first_scf_step": 4,
    "chfsi_iters_later_scf_steps": 1,
    "sre_tol_ry": 1e-4,
    "states": "roundup64(ceil(1.1 * n_electrons / 2))",
    "anderson_beta": 0.1,
    "anderson_history": 8,
    "poisson_cg_rtol": 1e-12,
    "multipole_lmax": 4,
    "lda": "PZ81 unpolarised",
    "bond_si_h_angstrom": 1.48,
    "lattice_angstrom": 5.43,
    "lattice_table_i_angstrom": 5.38,
}


def as_config() -> dict:
    """Every workload with its seeds, the model pseudopotential and the
    method constants, as one JSON-ready dictionary (written to
    synth/workloads.json by ``python -m synth.workloads``)."""
    import dataclasses
    wl = {}
    for name, w in WORKLOADS.items():
        d = dataclasses.asdict(w)
        d.update(geometry_seed=w.geometry_seed, x_seed=w.x_seed, lanczos_seed=w.lanczos_seed)
        wl[name] = d
    return {"workloads": wl, "model_pseudopotential": dataclasses.asdict(MODEL_PP), "method": dict(METHOD)}


if __name__ == "__main__":
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")
    with open(path, "w") as f:
        json.dump(as_config(), f, indent=1)
        f.write("\n")
    print(path)
