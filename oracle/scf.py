"""Oracle: the self-consistent field (SCF) loop around ChFSI.

Paper (computational details): LDA exchange-correlation in the Ceperley-
Alder form with the Perdew-Zunger parametrisation; four ChFSI iterations in
the first SCF step and one in each later step; convergence when the
self-consistent residual error (SRE) -- the square root of the density-
weighted integral of the squared difference of the last two potentials --
drops below 1e-4 Ry.

Readings where the paper is silent (all potentials in Ha, lengths in bohr):
* occupations f_i = 2 for the N_e / 2 lowest Ritz states, rho = sum f X^2 / h^3
  with X^T X = I; the output density of a step is scaled to hold N_e
  electrons (h^3 sum rho_out = N_e), which orthonormal columns give already;
* Hartree potential from the same 12th-order stencil, -L V = 4 pi rho on the
  inside points; stencil points outside the sphere take the multipole
  expansion (l <= 4, real solid harmonics about the grid origin) of rho;
  conjugate gradients to ||r|| / ||b|| < 1e-12 warm-started from the last V_H;
* PZ81 unpolarised LDA, eps_xc = v_xc = 0 where rho < 1e-14;
* SRE = 2 * sqrt(h^3 sum rho_out (V_Hxc[rho_out] - V_Hxc[rho_in])^2 / N_e) Ry;
* Anderson density mixing, history 6, beta = 0.3;
* Harris-Foulkes energy at rho_in:
  E = sum f eps - int rho (V_H + V_xc) + E_H + E_xc + E_II;
* initial density: superposition of Gaussian atoms Z (alpha / pi)^1.5
  exp(-alpha r^2), alpha_Si = 0.074, alpha_H = 0.21, renormalised to N_e;
* filter bounds: a = max, a0 = min Ritz value of the current subspace, b from
  10-step Lanczos on a fixed seeded vector; before the first Rayleigh-Ritz
  a0 = theta_min and a = theta_min + 0.1 (b - theta_min).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .chfsi import chebyshev_filter, cholesky_qr, lanczos_bound, rayleigh_ritz
from .grid import Grid, offsets
from .hamiltonian import Hamiltonian, fd_coefficients

RHO_MIN = 1e-14


# ----------------------------------------------------------------------------
# density and occupations
# ----------------------------------------------------------------------------
def density(X: np.ndarray, n_occ: int, h: float) -> np.ndarray:
    return 2.0 * (X[:, :n_occ] ** 2).sum(axis=1) / h ** 3


def sad_density(g: Grid, pos: np.ndarray, species: np.ndarray, n_electrons: int,
                alpha_si: float = 0.074, alpha_h: float = 0.21) -> np.ndarray:
    r = g.xyz
    rho = np.zeros(g.n)
    for a in range(len(species)):
        al = alpha_si if species[a] == 0 else alpha_h
        z = 4.0 if species[a] == 0 else 1.0
        d2 = ((r - pos[a]) ** 2).sum(axis=1)
        rho += z * (al / math.pi) ** 1.5 * np.exp(-al * d2)
    return rho * (n_electrons / (g.h ** 3 * rho.sum()))


# ----------------------------------------------------------------------------
# LDA (Perdew-Zunger 1981 fit of Ceperley-Alder, unpolarised)
# ----------------------------------------------------------------------------
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
EX_CONST = 0.75 * (9.0 / (4.0 * math.pi ** 2)) ** (1.0 / 3.0)   # eps_x = -EX_CONST / r_s


def lda_eps(rs: np.ndarray) -> np.ndarray:
    ex = -EX_CONST / rs
    sq = np.sqrt(rs)
    lnr = np.log(rs)
    ec = np.where(rs >= 1.0, PZ_GAMMA / (1.0 + PZ_BETA1 * sq + PZ_BETA2 * rs),
                  PZ_A * lnr + PZ_B + PZ_C * rs * lnr + PZ_D * rs)
    return ex + ec


def lda_deps_drs(rs: np.ndarray) -> np.ndarray:
    sq = np.sqrt(rs)
    lnr = np.log(rs)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * rs
    dec = np.where(rs >= 1.0, -PZ_GAMMA * (0.5 * PZ_BETA1 / sq + PZ_BETA2) / den ** 2,
                   PZ_A / rs + PZ_C * (lnr + 1.0) + PZ_D)
    return EX_CONST / rs ** 2 + dec


def lda(rho: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(eps_xc, v_xc) per point; v = eps - (r_s / 3) d eps / d r_s."""
    ok = rho >= RHO_MIN
    rs = (3.0 / (4.0 * math.pi * np.where(ok, rho, 1.0))) ** (1.0 / 3.0)
    eps = lda_eps(rs)
    v = eps - rs / 3.0 * lda_deps_drs(rs)
    return np.where(ok, eps, 0.0), np.where(ok, v, 0.0)


# ----------------------------------------------------------------------------
# Hartree potential
# ----------------------------------------------------------------------------
def solid_harmonics(x: np.ndarray, y: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Real regular solid harmonics R_lm = sqrt(4 pi / (2l+1)) r^l Y_lm, l <= 4,
    rows ordered l = 0..4 and within l: m = 0, then (cos, sin) for m = 1..l."""
    r2 = x * x + y * y + z * z
    s3, s5, s15 = math.sqrt(3.0), math.sqrt(5.0), math.sqrt(15.0)
    out = [np.ones_like(x),
           z, x, y,
           0.5 * (3 * z * z - r2), s3 * x * z, s3 * y * z, 0.5 * s3 * (x * x - y * y), s3 * x * y,
           0.5 * z * (5 * z * z - 3 * r2),
           math.sqrt(3 / 8) * x * (5 * z * z - r2), math.sqrt(3 / 8) * y * (5 * z * z - r2),
           0.5 * s15 * z * (x * x - y * y), s15 * x * y * z,
           math.sqrt(5 / 8) * x * (x * x - 3 * y * y), math.sqrt(5 / 8) * y * (3 * x * x - y * y),
           (35 * z ** 4 - 30 * z * z * r2 + 3 * r2 * r2) / 8.0,
           math.sqrt(10) / 4 * x * z * (7 * z * z - 3 * r2), math.sqrt(10) / 4 * y * z * (7 * z * z - 3 * r2),
           s5 / 4 * (x * x - y * y) * (7 * z * z - r2), s5 / 2 * x * y * (7 * z * z - r2),
           math.sqrt(70) / 4 * x * z * (x * x - 3 * y * y), math.sqrt(70) / 4 * y * z * (3 * x * x - y * y),
           math.sqrt(35) / 8 * (x ** 4 - 6 * x * x * y * y + y ** 4), math.sqrt(35) / 2 * x * y * (x * x - y * y)]
    return np.stack(out)


SH_L = np.array([0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3, 4, 4, 4, 4, 4, 4, 4, 4, 4])


def multipole_moments(g: Grid, rho: np.ndarray) -> np.ndarray:
    r = g.xyz
    return g.h ** 3 * solid_harmonics(r[:, 0], r[:, 1], r[:, 2]) @ rho


def multipole_potential(q: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Exterior potential sum_lm Q_lm R_lm(r) / r^(2l+1) at pts [K, 3]."""
    R = solid_harmonics(pts[:, 0], pts[:, 1], pts[:, 2])
    rr = np.sqrt((pts ** 2).sum(axis=1))
    return ((q[:, None] * R) / rr[None, :] ** (2 * SH_L[:, None] + 1)).sum(axis=0)


def ghost_points(g: Grid, nbr: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Stencil points outside the sphere: (owner rank, coefficient column k, coords)."""
    owners, ks, pts = [], [], []
    for col, (axis, k) in enumerate(offsets()):
        out = np.nonzero(nbr[:, col] < 0)[0]
        p = g.ijk[out].copy()
        p[:, axis] += k
        owners.append(out)
        ks.append(np.full(len(out), abs(k)))
        pts.append(p)
    return np.concatenate(owners), np.concatenate(ks), np.concatenate(pts).astype(np.float64) * g.h


def conjugate_gradient(apply_a, b: np.ndarray, x0: np.ndarray, rtol: float = 1e-12,
                       max_iter: int = 5000) -> tuple[np.ndarray, int]:
    x = x0.copy()
    r = b - apply_a(x)
    p = r.copy()
    rr = float(r @ r)
    bn = float(np.linalg.norm(b))
    it = 0
    while math.sqrt(rr) > rtol * bn and it < max_iter:
        ap = apply_a(p)
        alpha = rr / float(p @ ap)
        x += alpha * p
        r -= alpha * ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def hartree(g: Grid, lap, nbr: np.ndarray, rho: np.ndarray, v0: np.ndarray | None = None,
            rtol: float = 1e-12) -> tuple[np.ndarray, int]:
    owner, k, pts = ghost_points(g, nbr)
    vb = multipole_potential(multipole_moments(g, rho), pts)
    c = fd_coefficients() / (g.h * g.h)
    b = 4.0 * math.pi * rho + np.bincount(owner, weights=c[k] * vb, minlength=g.n)
    return conjugate_gradient(lambda v: -(lap @ v), b, np.zeros(g.n) if v0 is None else v0, rtol)


# ----------------------------------------------------------------------------
# mixing, SRE, energy
# ----------------------------------------------------------------------------
class Anderson:
    """Anderson mixing: minimise |F - dF gamma| over the history differences,
    then rho_next = (x - dX gamma) + beta (F - dF gamma)."""

    def __init__(self, beta: float = 0.3, history: int = 6):
        self.beta = beta
        self.history = history
        self.xs: list[np.ndarray] = []
        self.fs: list[np.ndarray] = []

    def mix(self, x: np.ndarray, f: np.ndarray) -> np.ndarray:
        if self.xs:
            dX = np.stack([x - xp for xp in self.xs], axis=1)
            dF = np.stack([f - fp for fp in self.fs], axis=1)
            gamma = np.linalg.solve(dF.T @ dF, dF.T @ f)
            xb, fb = x - dX @ gamma, f - dF @ gamma
        else:
            xb, fb = x, f
        self.xs.append(x.copy())
        self.fs.append(f.copy())
        if len(self.xs) > self.history:
            self.xs.pop(0)
            self.fs.pop(0)
        return xb + self.beta * fb


def sre_ry(h: float, rho_out: np.ndarray, dv: np.ndarray, n_electrons: int) -> float:
    return 2.0 * math.sqrt(h ** 3 * float((rho_out * dv * dv).sum()) / n_electrons)


def ion_energy(pos: np.ndarray, z: np.ndarray) -> float:
    e = 0.0
    for a in range(len(z)):
        d = np.sqrt(((pos[a + 1:] - pos[a]) ** 2).sum(axis=1))
        e += float((z[a] * z[a + 1:] / d).sum())
    return e


def harris_foulkes(h: float, eig: np.ndarray, n_occ: int, rho: np.ndarray, vh: np.ndarray,
                   eps_xc: np.ndarray, vxc: np.ndarray, e_ii: float) -> float:
    band = 2.0 * float(eig[:n_occ].sum())
    h3 = h ** 3
    return band - h3 * float(rho @ (vh + vxc)) + 0.5 * h3 * float(rho @ vh) + h3 * float(rho @ eps_xc) + e_ii


# ----------------------------------------------------------------------------
# SCF driver
# ----------------------------------------------------------------------------
@dataclass
class ScfState:
    rho_in: np.ndarray
    X: np.ndarray
    vh: np.ndarray
    a: float | None = None
    a0: float | None = None
    step: int = 0
    mixer: Anderson = field(default_factory=Anderson)


@dataclass
class ScfReport:
    step: int
    sre_ry: float
    energy: float
    eig: np.ndarray
    homo: float
    lumo: float
    b: float
    cg_iters: int


def scf_step(H: Hamiltonian, nbr: np.ndarray, st: ScfState, n_electrons: int, degree: int,
             v_lanczos: np.ndarray, e_ii: float, lanczos_k: int = 10) -> ScfReport:
    g = H.grid
    n_occ = n_electrons // 2
    st.step += 1
    vh_in, it1 = hartree(g, H.lap, nbr, st.rho_in, st.vh)
    exc_in, vxc_in = lda(st.rho_in)
    H.veff = H.vloc + vh_in + vxc_in
    b, tmin, _ = lanczos_bound(H.apply, v_lanczos, lanczos_k)
    if st.a is None:
        st.a0 = tmin
        st.a = tmin + 0.1 * (b - tmin)
    X = st.X
    lam = None
    for _ in range(4 if st.step == 1 else 1):
        Y = chebyshev_filter(H.apply, X, degree, st.a, b, st.a0)
        Q, _ = cholesky_qr(Y)
        lam, X = rayleigh_ritz(H.apply, Q)
        st.a, st.a0 = float(lam[-1]), float(lam[0])
    st.X = X
    rho_out = density(X, n_occ, g.h)
    rho_out *= n_electrons / (g.h ** 3 * float(rho_out.sum()))
    vh_out, it2 = hartree(g, H.lap, nbr, rho_out, vh_in)
    _, vxc_out = lda(rho_out)
    sre = sre_ry(g.h, rho_out, (vh_out + vxc_out) - (vh_in + vxc_in), n_electrons)
    energy = harris_foulkes(g.h, lam, n_occ, st.rho_in, vh_in, exc_in, vxc_in, e_ii)
    st.rho_in = st.mixer.mix(st.rho_in, rho_out - st.rho_in)
    st.vh = vh_in
    return ScfReport(st.step, sre, energy, lam, float(lam[n_occ - 1]), float(lam[n_occ]), b, it1 + it2)
