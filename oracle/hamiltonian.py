"""Oracle: the real-space Kohn-Sham Hamiltonian on the spherical grid.

Paper: the Kohn-Sham equations are discretised by high-order finite
differences in real space (the PARSEC description); the pseudopotentials are
norm-conserving in Kleinman-Bylander separable form (computational details);
H is large and very sparse.

    H = -1/2 L + diag(V_eff) + sum_a sum_lm |beta_alm> h_l <beta_alm|

Readings where the paper is silent:
* L is the 12th-order central second-difference stencil applied along x, y
  and z (13 points per axis, 37-point star), coefficients from Fornberg's
  closed form; psi = 0 at every grid point outside the sphere;
* V_loc(r) = -sum_a Z_a erf(|r - R_a| / r_loc) / |r - R_a| with Z_Si = 4,
  Z_H = 1, r_loc = 0.7 bohr for Si and 0.5 bohr for H, and the r -> 0 limit
  -2 Z / (sqrt(pi) r_loc) (with a 0.9 bohr H width the Si-H bonds are so weak
  that no HOMO-LUMO gap forms in the smallest cluster; with a 0.9 bohr Si
  width the gap closes by 3 nm);
* one s and one p Gaussian projector per Si in the Goedecker-Teter-Hutter
  form p_l(r) = N_l r^l exp(-r^2 / (2 r_c^2)), r_c = 1.2 bohr, normalised by
  int p_l^2 r^2 dr = 1, times real harmonics, cut at |r - R_a| <= 4.8 bohr;
  KB energies h_s = 3.0 Ha, h_p = 0.0 Ha by default (chosen so that clusters
  from 0.55 to 4 nm converge with an open gap); H atoms carry no projector;
* <beta|X> is the quadrature h^3 sum_q beta(q) X(q).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
from scipy.special import erf

from .grid import Grid, HALF_ORDER, neighbour_table, offsets


@dataclass
class PseudoParams:
    z_si: float = 4.0
    z_h: float = 1.0
    r_loc: float = 0.7
    r_loc_h: float = 0.5
    r_c: float = 1.2
    r_cut: float = 4.8
    h_s: float = 3.0
    h_p: float = 0.0

    def charges(self, species: np.ndarray) -> np.ndarray:
        return np.where(species == 0, self.z_si, self.z_h).astype(np.float64)

    def widths(self, species: np.ndarray) -> np.ndarray:
        return np.where(species == 0, self.r_loc, self.r_loc_h).astype(np.float64)


def fd_coefficients_exact(p: int = HALF_ORDER) -> list[Fraction]:
    """Central 2p-order second-derivative weights c_0..c_p (Fornberg's closed form)."""
    c = [Fraction(0)] * (p + 1)
    for k in range(1, p + 1):
        c[k] = Fraction(2 * (-1) ** (k + 1) * math.factorial(p) ** 2,
                        k * k * math.factorial(p - k) * math.factorial(p + k))
    c[0] = -2 * sum(c[1:])
    return c


def fd_coefficients(p: int = HALF_ORDER) -> np.ndarray:
    return np.array([float(x) for x in fd_coefficients_exact(p)])


def laplacian(g: Grid, nbr: np.ndarray | None = None) -> sp.csr_matrix:
    """Zero-padded FD Laplacian on the grid, rank order, CSR."""
    if nbr is None:
        nbr = neighbour_table(g)
    c = fd_coefficients() / (g.h * g.h)
    rows = [np.arange(g.n)]
    cols = [np.arange(g.n)]
    vals = [np.full(g.n, 3.0 * c[0])]
    for col, (_axis, k) in enumerate(offsets()):
        ok = nbr[:, col] >= 0
        rows.append(np.nonzero(ok)[0])
        cols.append(nbr[ok, col].astype(np.int64))
        vals.append(np.full(int(ok.sum()), c[abs(k)]))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.n, g.n))


def local_potential(g: Grid, pos: np.ndarray, species: np.ndarray, pp: PseudoParams) -> np.ndarray:
    """V_loc at every grid point (rank order): erf-screened point charges."""
    r = g.xyz
    z = pp.charges(species)
    w = pp.widths(species)
    v = np.zeros(g.n)
    for a in range(len(z)):
        d = np.sqrt(((r - pos[a]) ** 2).sum(axis=1))
        small = d < 1e-8
        dd = np.where(small, 1.0, d)
        v -= np.where(small, 2.0 * z[a] / (math.sqrt(math.pi) * w[a]), z[a] * erf(dd / w[a]) / dd)
    return v


def projector_matrix(g: Grid, pos: np.ndarray, species: np.ndarray, pp: PseudoParams) -> tuple[sp.csc_matrix, np.ndarray]:
    """B [N, 4 N_Si] with columns (atom; s, px, py, pz) and the KB energies per column."""
    r = g.xyz
    n_s = math.sqrt(4.0 / (math.sqrt(math.pi) * pp.r_c ** 3))
    n_p = math.sqrt(8.0 / (3.0 * math.sqrt(math.pi) * pp.r_c ** 5))
    y00 = 1.0 / math.sqrt(4.0 * math.pi)
    y1 = math.sqrt(3.0 / (4.0 * math.pi))
    rows, cols, vals, energies = [], [], [], []
    col = 0
    for a in np.nonzero(species == 0)[0]:
        dx = r[:, 0] - pos[a, 0]
        dy = r[:, 1] - pos[a, 1]
        dz = r[:, 2] - pos[a, 2]
        d2 = dx * dx + dy * dy + dz * dz
        sup = np.nonzero(d2 <= pp.r_cut * pp.r_cut)[0]
        gauss = np.exp(-d2[sup] / (2.0 * pp.r_c * pp.r_c))
        for lm, f in enumerate((n_s * y00 * gauss, n_p * y1 * gauss * dx[sup],
                                n_p * y1 * gauss * dy[sup], n_p * y1 * gauss * dz[sup])):
            rows.append(sup)
            cols.append(np.full(len(sup), col + lm))
            vals.append(f)
        energies += [pp.h_s, pp.h_p, pp.h_p, pp.h_p]
        col += 4
    B = sp.csc_matrix((np.concatenate(vals) if vals else np.zeros(0),
                       (np.concatenate(rows) if rows else np.zeros(0, np.int64),
                        np.concatenate(cols) if cols else np.zeros(0, np.int64))), shape=(g.n, col))
    return B, np.array(energies)


@dataclass
class Hamiltonian:
    grid: Grid
    lap: sp.csr_matrix       # L (not -1/2 L)
    vloc: np.ndarray
    veff: np.ndarray
    B: sp.csc_matrix
    kb_energy: np.ndarray

    def apply(self, X: np.ndarray) -> np.ndarray:
        """H X for X [N, M] (or [N]) in rank order."""
        h3 = self.grid.h ** 3
        v = self.veff if X.ndim == 1 else self.veff[:, None]
        Y = -0.5 * (self.lap @ X) + v * X
        if self.B.shape[1]:
            C = h3 * (self.B.T @ X)
            Y = Y + self.B @ ((self.kb_energy if X.ndim == 1 else self.kb_energy[:, None]) * C)
        return Y

    def dense(self) -> np.ndarray:
        """Dense H (tiny grids only)."""
        H = -0.5 * self.lap.toarray() + np.diag(self.veff)
        if self.B.shape[1]:
            Bd = self.B.toarray()
            H += self.grid.h ** 3 * (Bd * self.kb_energy) @ Bd.T
        return H


def build_hamiltonian(g: Grid, pos: np.ndarray, species: np.ndarray, pp: PseudoParams | None = None,
                      with_vloc: bool = True) -> Hamiltonian:
    pp = pp or PseudoParams()
    lap = laplacian(g)
    vloc = local_potential(g, pos, species, pp) if with_vloc else np.zeros(g.n)
    B, e = projector_matrix(g, pos, species, pp)
    return Hamiltonian(g, lap, vloc, vloc.copy(), B, e)


def apply_at_points(ijk: np.ndarray, x_at, h: float, radius: float, pos: np.ndarray, species: np.ndarray,
                    pp: PseudoParams, veff: np.ndarray | None = None) -> np.ndarray:
    """(H X)(p) at the integer grid points ``ijk`` [P, 3], one point at a time,
    for sizes where the whole-grid operator cannot be assembled.

    ``x_at(pts)`` returns the rows of X [len(pts), M] at integer points
    ``pts`` that lie inside the sphere (the caller's layout lookup).  The
    terms are the definitions above: the 37-point star of -1/2 L with zero
    values outside the sphere, V_eff (V_loc when ``veff`` is None) times X,
    and for every Si atom within r_cut of p the KB term
    sum_lm h_l beta_alm(p) C_alm with C_alm = h^3 sum_q beta_alm(q) X(q) over
    the atom's support points q inside the sphere.
    Returns (HX [P, M], magnitude [P, M]): the second is the sum of the
    absolute values of the terms, the scale of the rounding error of any
    evaluation of the same sum.
    """
    n_r = int(math.floor(radius / h))
    thr = math.floor((radius / h) ** 2 + 1e-9)

    def inside(p):
        return (p * p).sum(axis=-1) <= thr

    c = fd_coefficients() / (h * h)
    n_s = math.sqrt(4.0 / (math.sqrt(math.pi) * pp.r_c ** 3))
    n_p = math.sqrt(8.0 / (3.0 * math.sqrt(math.pi) * pp.r_c ** 5))
    y00 = 1.0 / math.sqrt(4.0 * math.pi)
    y1 = math.sqrt(3.0 / (4.0 * math.pi))
    si = np.nonzero(species == 0)[0]
    z = pp.charges(species)
    w = pp.widths(species)
    kcut = int(math.ceil(pp.r_cut / h)) + 1
    out, mag = [], []
    for p in np.asarray(ijk, dtype=np.int64):
        xp = x_at(p[None])[0]
        y = np.zeros_like(xp, dtype=np.float64)
        a_sum = np.zeros_like(y)
        # -1/2 L: centre weight appears once per axis
        y += -0.5 * 3.0 * c[0] * xp
        a_sum += abs(1.5 * c[0]) * np.abs(xp)
        for axis in range(3):
            for k in range(1, HALF_ORDER + 1):
                for sgn in (-1, 1):
                    q = p.copy()
                    q[axis] += sgn * k
                    if inside(q):
                        xq = x_at(q[None])[0]
                        y += -0.5 * c[k] * xq
                        a_sum += abs(0.5 * c[k]) * np.abs(xq)
        r = p.astype(np.float64) * h
        if veff is None:
            d = np.sqrt(((pos - r) ** 2).sum(axis=1))
            small = d < 1e-8
            dd = np.where(small, 1.0, d)
            v = -float(np.where(small, 2.0 * z / (math.sqrt(math.pi) * w), z * erf(dd / w) / dd).sum())
        else:
            v = float(veff)
        y += v * xp
        a_sum += abs(v) * np.abs(xp)
        for a in si:
            dv = r - pos[a]
            if float(dv @ dv) > pp.r_cut ** 2:
                continue
            # the atom's support: grid points within r_cut of it, inside the sphere
            ca = np.round(pos[a] / h).astype(np.int64)
            g = np.arange(-kcut, kcut + 1)
            gi, gj, gk = np.meshgrid(g, g, g, indexing="ij")
            pts = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1) + ca
            rel = pts.astype(np.float64) * h - pos[a]
            d2 = (rel * rel).sum(axis=1)
            keep = (d2 <= pp.r_cut ** 2) & inside(pts)
            pts, rel, d2 = pts[keep], rel[keep], d2[keep]
            gq = np.exp(-d2 / (2.0 * pp.r_c ** 2))
            bq = np.stack([n_s * y00 * gq, n_p * y1 * gq * rel[:, 0], n_p * y1 * gq * rel[:, 1],
                           n_p * y1 * gq * rel[:, 2]], axis=1)
            xq = x_at(pts)
            cq = h ** 3 * (bq.T @ xq)
            gp = math.exp(-float(dv @ dv) / (2.0 * pp.r_c ** 2))
            bp = np.array([n_s * y00 * gp, n_p * y1 * gp * dv[0], n_p * y1 * gp * dv[1], n_p * y1 * gp * dv[2]])
            hl = np.array([pp.h_s, pp.h_p, pp.h_p, pp.h_p])
            y += (bp * hl) @ cq
            a_sum += np.abs(bp * hl) @ (h ** 3 * (np.abs(bq).T @ np.abs(xq)))
        out.append(y)
        mag.append(a_sum)
    return np.array(out), np.array(mag)
