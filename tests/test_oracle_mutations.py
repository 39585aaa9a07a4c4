"""Planted mistakes in the oracle, on the CPU.

Each case patches one plausible slip into one oracle function (a dropped
term or factor, a flipped sign, a wrong index or axis, a transposed
operand) and runs the committed pins that cover that function; at least one
of them must fail.  This shows that the pins constrain the oracle beyond
restating its formulas.  The mistakes live only in this file, as wrong
copies or wrappers of oracle functions; nothing here touches the HIP path.
"""
import dataclasses
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.special import erf

from oracle import chfsi as C
from oracle import grid as G
from oracle import hamiltonian as OH
from oracle import scf as S
from oracle import unet as U

import oracle_systems
import test_oracle_chfsi as TC
import test_oracle_grid as TG
import test_oracle_hamiltonian as TH
import test_oracle_scf as TS
import test_oracle_unet as TU

# the oracle as written, for wrappers that plant a slip around it
LANCZOS = C.lanczos_bound
LAPLACIAN = OH.laplacian
PROJECTORS = OH.projector_matrix
HILBERT = G.hilbert_index3
CONV3D = U.conv3d
POINTWISE = OH.apply_at_points
SOLID = S.solid_harmonics


# ---------------------------------------------------------------------------
# Chebyshev filter, Lanczos bound, Cholesky-QR, Rayleigh-Ritz
# ---------------------------------------------------------------------------
def filter_scalars_beta_squared(m, a, b, a0):
    e, c = (b - a) / 2.0, (b + a) / 2.0
    s1 = e / (a0 - c)
    out, s = [(s1 / e, c, 0.0)], s1
    for _ in range(2, m + 1):
        sn = 1.0 / (2.0 / s1 - s)
        out.append((2.0 * sn / e, c, sn * sn))          # slip: sigma_{k+1}^2 for sigma_k sigma_{k+1}
        s = sn
    return out


def filter_scalars_sigma1_sign(m, a, b, a0):
    e, c = (b - a) / 2.0, (b + a) / 2.0
    s1 = e / (c - a0)                                    # slip: sign of sigma_1
    out, s = [(s1 / e, c, 0.0)], s1
    for _ in range(2, m + 1):
        sn = 1.0 / (2.0 / s1 - s)
        out.append((2.0 * sn / e, c, s * sn))
        s = sn
    return out


def filter_without_shift(apply_h, X, m, a, b, a0):
    prev = cur = X
    for k, (alpha, c, beta) in enumerate(C.filter_scalars(m, a, b, a0)):
        nxt = alpha * apply_h(cur)                       # slip: (H - c) Y became H Y
        if k > 0:
            nxt = nxt - beta * prev
        prev, cur = cur, nxt
    return cur


def filter_h_on_older_iterate(apply_h, X, m, a, b, a0):
    prev = cur = X
    for k, (alpha, c, beta) in enumerate(C.filter_scalars(m, a, b, a0)):
        nxt = alpha * (apply_h(prev) - c * cur)          # slip: H applied to Y_{k-2}
        if k > 0:
            nxt = nxt - beta * prev
        prev, cur = cur, nxt
    return cur


def lanczos_without_residual(apply_h, v0, k=10):
    _, tmin, tmax = LANCZOS(apply_h, v0, k)
    return tmax, tmin, tmax                              # slip: the bound misses ||f_k||


def cholesky_qr_lower_factor(X):
    R = np.linalg.cholesky(X.T @ X)                      # slip: the lower factor taken as R
    return np.linalg.solve(R.T, X.T).T, R


def rayleigh_ritz_rotation_transposed(apply_h, X):
    Hs = X.T @ apply_h(X)
    lam, Q = np.linalg.eigh(0.5 * (Hs + Hs.T))
    return lam, X @ Q.T                                  # slip: rotated by Q^T


def rayleigh_ritz_without_h(apply_h, X):
    Hs = X.T @ X                                         # slip: the Gram matrix for X^T H X
    lam, Q = np.linalg.eigh(0.5 * (Hs + Hs.T))
    return lam, X @ Q


# ---------------------------------------------------------------------------
# Hamiltonian
# ---------------------------------------------------------------------------
def fd_weights_sign(p=6):
    c = [Fraction(0)] * (p + 1)
    for k in range(1, p + 1):
        c[k] = Fraction(2 * (-1) ** k * math.factorial(p) ** 2,     # slip: (-1)^k for (-1)^(k+1)
                        k * k * math.factorial(p - k) * math.factorial(p + k))
    c[0] = -2 * sum(c[1:])
    return c


def laplacian_centre_once(g, nbr=None):
    c0 = OH.fd_coefficients()[0] / g.h ** 2
    return (LAPLACIAN(g, nbr) - (2.0 * c0) * sp.identity(g.n, format="csr")).tocsr()   # slip: c_0 once, not per axis


def laplacian_over_h(g, nbr=None):
    return (g.h * LAPLACIAN(g, nbr)).tocsr()             # slip: weights divided by h, not h^2

def laplacian_signed_index(g, nbr=None):
    if nbr is None:
        nbr = G.neighbour_table(g)
    c = OH.fd_coefficients() / (g.h * g.h)
    rows, cols, vals = [np.arange(g.n)], [np.arange(g.n)], [np.full(g.n, 3.0 * c[0])]
    for col, (_axis, k) in enumerate(G.offsets()):
        ok = nbr[:, col] >= 0
        rows.append(np.nonzero(ok)[0])
        cols.append(nbr[ok, col].astype(np.int64))
        vals.append(np.full(int(ok.sum()), c[k]))        # slip: c[k] for c[|k|] (negative k wraps)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(g.n, g.n))


def _vloc(g, pos, species, pp, limit_factor, arg):
    z, w = pp.charges(species), pp.widths(species)
    v = np.zeros(g.n)
    for a in range(len(z)):
        d = np.sqrt(((g.xyz - pos[a]) ** 2).sum(axis=1))
        small = d < 1e-8
        dd = np.where(small, 1.0, d)
        v -= np.where(small, limit_factor * z[a] / (math.sqrt(math.pi) * w[a]), z[a] * erf(arg(dd, w[a])) / dd)
    return v


def vloc_limit_without_2(g, pos, species, pp):
    return _vloc(g, pos, species, pp, 1.0, lambda d, w: d / w)      # slip: the r -> 0 limit loses its 2


def vloc_erf_argument(g, pos, species, pp):
    return _vloc(g, pos, species, pp, 2.0, lambda d, w: d * w)      # slip: erf(d r_loc) for erf(d / r_loc)


def projectors_p_norm(g, pos, species, pp):
    B, e = PROJECTORS(g, pos, species, pp)
    # slip: N_p with r_c^3 in place of r_c^5 (the p columns come out r_c times too large)
    scale = np.tile([1.0, pp.r_c, pp.r_c, pp.r_c], B.shape[1] // 4)
    return (B @ sp.diags(scale)).tocsc(), e


def _apply(self, X, kinetic, h3):
    v = self.veff if X.ndim == 1 else self.veff[:, None]
    Y = kinetic * (self.lap @ X) + v * X
    if self.B.shape[1]:
        e = self.kb_energy if X.ndim == 1 else self.kb_energy[:, None]
        Y = Y + self.B @ (e * (h3(self) * (self.B.T @ X)))
    return Y


def apply_kb_without_h3(self, X):
    return _apply(self, X, -0.5, lambda H: 1.0)                     # slip: quadrature weight h^3 dropped


def apply_kinetic_sign(self, X):
    return _apply(self, X, 0.5, lambda H: H.grid.h ** 3)            # slip: +1/2 L for -1/2 L


def pointwise_without_kb(ijk, x_at, h, radius, pos, species, pp, veff=None):
    no_kb = dataclasses.replace(pp, h_s=0.0, h_p=0.0)   # slip: KB term dropped
    return POINTWISE(ijk, x_at, h, radius, pos, species, no_kb, veff)


# ---------------------------------------------------------------------------
# grid, Hilbert order, neighbours
# ---------------------------------------------------------------------------
def hilbert_without_gray_decode(x, y, z, nbits):
    X = [np.asarray(x, np.int64).copy(), np.asarray(y, np.int64).copy(), np.asarray(z, np.int64).copy()]
    top = 1 << (nbits - 1)
    q = top
    while q > 1:
        p = q - 1
        for i in range(3):
            hit = (X[i] & q) != 0
            X[0] = np.where(hit, X[0] ^ p, X[0])
            t = np.where(hit, 0, (X[0] ^ X[i]) & p)
            X[0] = X[0] ^ t
            X[i] = X[i] ^ t
        q >>= 1
    # slip: the Gray encoding across axes (X[1] ^= X[0], X[2] ^= X[1] and the
    # correction word) is left out
    idx = np.zeros_like(X[0])
    for lvl in range(nbits - 1, -1, -1):
        for i in range(3):
            idx = (idx << 1) | ((X[i] >> lvl) & 1)
    return idx


def hilbert_z_first(x, y, z, nbits):
    return HILBERT(z, y, x, nbits)                       # slip: bits interleaved z first


def hilbert_bits_of_count(n_blocks_edge):
    return max(1, int(n_blocks_edge).bit_length())    # slip: bits of n, not of n - 1

def sphere_points_strict(radius, h):
    n_r = int(math.floor(radius / h))
    thr = math.floor((radius / h) ** 2 + 1e-9)
    g = np.arange(-n_r, n_r + 1, dtype=np.int64)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    inside = (i * i + j * j + k * k) < thr               # slip: points on the sphere dropped
    return n_r, np.stack([i[inside], j[inside], k[inside]], axis=1)


def neighbour_table_sign(g):
    n = 2 * g.n_r + 1
    cube = -np.ones((n, n, n), dtype=np.int64)
    I = g.ijk + g.n_r
    cube[I[:, 0], I[:, 1], I[:, 2]] = np.arange(g.n)
    out = -np.ones((g.n, 36), dtype=np.int64)
    for c, (axis, k) in enumerate(G.offsets()):
        J = I.copy()
        J[:, axis] -= k                                  # slip: offset applied with the wrong sign
        ok = (J[:, axis] >= 0) & (J[:, axis] < n)
        out[ok, c] = cube[J[ok, 0], J[ok, 1], J[ok, 2]]
    return out.astype(np.int32)


def build_grid_local_xy_swapped(radius, h, ordering=G.ORDER_HILBERT):
    n_r, pts = G.sphere_points(radius, h)
    if ordering == G.ORDER_LEX:
        order = np.lexsort((pts[:, 0], pts[:, 1], pts[:, 2]))
        ijk = pts[order]
        return G.Grid(h, radius, n_r, ijk, np.arange(len(ijk), dtype=np.int64), len(ijk), ordering,
                      np.zeros((0, 3), np.int64))
    I = pts + n_r
    B = I // G.BLOCK
    nb = (2 * n_r) // G.BLOCK + 1
    key = G.hilbert_index3(B[:, 0], B[:, 1], B[:, 2], G.hilbert_bits(nb))
    ukey, first = np.unique(key, return_index=True)
    slot = np.searchsorted(ukey, key)
    local = (I[:, 1] % G.BLOCK) + G.BLOCK * (I[:, 0] % G.BLOCK) + G.BLOCK ** 2 * (I[:, 2] % G.BLOCK)   # slip: y fastest
    row = slot * G.BLOCK ** 3 + local
    order = np.argsort(row, kind="stable")
    return G.Grid(h, radius, n_r, pts[order], row[order], len(ukey) * G.BLOCK ** 3, ordering, B[first])


def offsets_positive_first():
    return [(axis, k) for axis in range(3) for k in list(range(1, 7)) + list(range(-6, 0))]   # slip: +k before -k


# ---------------------------------------------------------------------------
# SCF pieces
# ---------------------------------------------------------------------------
def lda_potential_sign(rho):
    ok = rho >= S.RHO_MIN
    rs = (3.0 / (4.0 * math.pi * np.where(ok, rho, 1.0))) ** (1.0 / 3.0)
    eps = S.lda_eps(rs)
    v = eps + rs / 3.0 * S.lda_deps_drs(rs)              # slip: + (r_s / 3) d eps / d r_s
    return np.where(ok, eps, 0.0), np.where(ok, v, 0.0)


def anderson_extrapolation_sign(self, x, f):
    if self.xs:
        dX = np.stack([x - xp for xp in self.xs], axis=1)
        dF = np.stack([f - fp for fp in self.fs], axis=1)
        gamma = np.linalg.solve(dF.T @ dF, dF.T @ f)
        xb, fb = x + dX @ gamma, f - dF @ gamma          # slip: + dX gamma
    else:
        xb, fb = x, f
    self.xs.append(x.copy())
    self.fs.append(f.copy())
    if len(self.xs) > self.history:
        self.xs.pop(0)
        self.fs.pop(0)
    return xb + self.beta * fb


def _harris_foulkes(occ, hartree, xc_dc):
    def hf(h, eig, n_occ, rho, vh, eps_xc, vxc, e_ii):
        h3 = h ** 3
        return (occ * float(eig[:n_occ].sum()) - h3 * float(rho @ (vh + xc_dc * vxc))
                + hartree * h3 * float(rho @ vh) + h3 * float(rho @ eps_xc) + e_ii)
    return hf


def density_single_occupation(X, n_occ, h):
    return (X[:, :n_occ] ** 2).sum(axis=1) / h ** 3      # slip: one electron per state


def density_without_h3(X, n_occ, h):
    return 2.0 * (X[:, :n_occ] ** 2).sum(axis=1)         # slip: grid normalisation dropped


def sre_in_hartree(h, rho_out, dv, n_electrons):
    return math.sqrt(h ** 3 * float((rho_out * dv * dv).sum()) / n_electrons)   # slip: Hartree, not Rydberg


def sre_without_root(h, rho_out, dv, n_electrons):
    return 2.0 * h ** 3 * float((rho_out * dv * dv).sum()) / n_electrons       # slip: mean square, no root

def ion_energy_all_ordered_pairs(pos, z):
    e = 0.0
    for a in range(len(z)):
        d = np.sqrt(((pos - pos[a]) ** 2).sum(axis=1))
        d[a] = np.inf
        e += float((z[a] * z / d).sum())                 # slip: every pair counted twice
    return e


def lda_derivative_branch(rs):
    sq, lnr = np.sqrt(rs), np.log(rs)
    den = 1.0 + S.PZ_BETA1 * sq + S.PZ_BETA2 * rs
    dec = np.where(rs >= 1.0, -S.PZ_GAMMA * (0.5 * S.PZ_BETA1 / sq + S.PZ_BETA2) / den ** 2,
                   S.PZ_A / rs + S.PZ_C * lnr + S.PZ_D)   # slip: d(C r ln r)/dr taken as C ln r
    return S.EX_CONST / rs ** 2 + dec


def sad_density_unnormalised(g, pos, species, n_electrons, alpha_si=0.074, alpha_h=0.21):
    rho = np.zeros(g.n)
    for a in range(len(species)):
        al = alpha_si if species[a] == 0 else alpha_h
        z = 4.0 if species[a] == 0 else 1.0
        rho += z * (al / math.pi) ** 1.5 * np.exp(-al * ((g.xyz - pos[a]) ** 2).sum(axis=1))
    return rho * (n_electrons / rho.sum())                # slip: h^3 left out of the normalisation


def _sad_with(z_si, z_h, swap, half_exponent, norm_power):
    def sad(g, pos, species, n_electrons, alpha_si=0.074, alpha_h=0.21):
        rho = np.zeros(g.n)
        for a in range(len(species)):
            si = species[a] == 0
            al = (alpha_h if si else alpha_si) if swap else (alpha_si if si else alpha_h)
            z = z_si if si else z_h
            d2 = ((g.xyz - pos[a]) ** 2).sum(axis=1)
            rho += z * (al / math.pi) ** norm_power * np.exp(-(0.5 if half_exponent else 1.0) * al * d2)
        return rho * (n_electrons / (g.h ** 3 * rho.sum()))
    return sad


sad_density_widths_swapped = _sad_with(4.0, 1.0, True, False, 1.5)        # slip: alpha_Si and alpha_H exchanged
sad_density_half_exponent = _sad_with(4.0, 1.0, False, True, 1.5)         # slip: exp(-alpha r^2 / 2)
sad_density_norm_power_one = _sad_with(4.0, 1.0, False, False, 1.0)       # slip: (alpha / pi)^1
sad_density_equal_charges = _sad_with(1.0, 1.0, False, False, 1.5)        # slip: Z = 1 for Si


def solid_harmonics_unscaled_l2(x, y, z):
    R = SOLID(x, y, z).copy()
    R[4] *= 2.0                                          # slip: (3 z^2 - r^2) without its 1/2
    return R


def multipole_moments_without_h3(g, rho):
    r = g.xyz
    return S.solid_harmonics(r[:, 0], r[:, 1], r[:, 2]) @ rho   # slip: quadrature weight dropped


def multipole_potential_exponent(q, pts):
    R = S.solid_harmonics(pts[:, 0], pts[:, 1], pts[:, 2])
    rr = np.sqrt((pts ** 2).sum(axis=1))
    return ((q[:, None] * R) / rr[None, :] ** (2 * S.SH_L[:, None])).sum(axis=0)   # slip: r^(2l) for r^(2l+1)


def ghost_points_signed_k(g, nbr):
    owners, ks, pts = [], [], []
    for col, (axis, k) in enumerate(G.offsets()):
        out = np.nonzero(nbr[:, col] < 0)[0]
        p = g.ijk[out].copy()
        p[:, axis] += k
        owners.append(out)
        ks.append(np.full(len(out), k))                  # slip: signed k as the weight index
        pts.append(p)
    return np.concatenate(owners), np.concatenate(ks), np.concatenate(pts).astype(np.float64) * g.h


def cg_beta_inverted(apply_a, b, x0, rtol=1e-12, max_iter=5000):
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
        p = r + (rr / rr_new) * p                        # slip: beta = |r_k|^2 / |r_k+1|^2
        rr = rr_new
        it += 1
    return x, it


def hartree_source_without_4pi(g, lap, nbr, rho, v0=None, rtol=1e-12):
    owner, k, pts = S.ghost_points(g, nbr)
    vb = S.multipole_potential(S.multipole_moments(g, rho), pts)
    c = OH.fd_coefficients() / (g.h * g.h)
    b = rho + np.bincount(owner, weights=c[k] * vb, minlength=g.n)   # slip: 4 pi rho written as rho
    return S.conjugate_gradient(lambda v: -(lap @ v), b, np.zeros(g.n) if v0 is None else v0, rtol)


def hartree_boundary_sign(g, lap, nbr, rho, v0=None, rtol=1e-12):
    owner, k, pts = S.ghost_points(g, nbr)
    vb = S.multipole_potential(S.multipole_moments(g, rho), pts)
    c = OH.fd_coefficients() / (g.h * g.h)
    b = 4.0 * math.pi * rho - np.bincount(owner, weights=c[k] * vb, minlength=g.n)   # slip: boundary term subtracted
    return S.conjugate_gradient(lambda v: -(lap @ v), b, np.zeros(g.n) if v0 is None else v0, rtol)


# ---------------------------------------------------------------------------
# density network
# ---------------------------------------------------------------------------
def conv_flipped_kernel(x, w, b, stride=1):
    return CONV3D(x, np.ascontiguousarray(w[:, :, ::-1, ::-1, ::-1]), b, stride)   # slip: convolution for correlation


def silu_grad_first_term_only(z):
    return 1.0 / (1.0 + np.exp(-z))                      # slip: sigma(z) for sigma(z)(1 + z(1 - sigma(z)))


def mse_sum(y, t):
    diff = y - t
    return float((diff * diff).sum()), 2.0 * diff     # slip: sum for mean (loss and gradient agree)

def adam_without_bias_correction(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        p[k] = p[k] - lr * m[k] / (np.sqrt(v[k]) + eps)  # slip: no 1 / (1 - b^t) corrections


def upsample_backward_mean(dy):
    C_, D, H, W = dy.shape
    return dy.reshape(C_, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))   # slip: mean for sum


def conv_backward_dw_shift(x, w, dy, stride=1):
    k = w.shape[2]
    pad = k // 2
    D, H, W = x.shape[1:]
    if stride == 2:
        full = np.zeros((dy.shape[0], D, H, W))
        full[:, ::2, ::2, ::2] = dy
        dy = full
    db = dy.sum(axis=(1, 2, 3))
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad)))
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for dz in range(k):
        for dy_ in range(k):
            for dx in range(k):
                sl = xp[:, k - 1 - dz:k - 1 - dz + D, dy_:dy_ + H, dx:dx + W]   # slip: tap z mirrored in dW
                dw[:, :, dz, dy_, dx] = np.einsum("odhw,idhw->oi", dy, sl)
                dxp[:, dz:dz + D, dy_:dy_ + H, dx:dx + W] += np.einsum("oi,odhw->idhw", w[:, :, dz, dy_, dx], dy)
    return dxp[:, pad:pad + D, pad:pad + H, pad:pad + W], dw, db


def highpass_unnormalised(box, sigma):
    r = int(math.ceil(3.0 * sigma))
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-k * k / (2.0 * sigma * sigma))           # slip: weights not normalised to unit sum
    out = np.asarray(box, dtype=np.float64)
    for axis in range(3):
        out = np.apply_along_axis(lambda v: np.convolve(v, g, mode="same"), axis, out)
    return np.asarray(box, dtype=np.float64) - out


# ---------------------------------------------------------------------------
# the pins each slip is run against
# ---------------------------------------------------------------------------
PINS = {
    "filter = polynomial on eigenpairs": lambda f: TC.test_filter_equals_polynomial_on_eigenpairs(f["tiny"]),
    "filter scalars = Chebyshev ratios": lambda f: TC.test_filter_scalars_are_chebyshev_ratios(12, 0.1, 40.0, -0.5),
    "filter normalisation": lambda f: TC.test_filter_scalars_normalisation(),
    "Lanczos upper bound": lambda f: TC.test_lanczos_upper_bound(f["tiny"]),
    "Cholesky-QR = Householder": lambda f: TC.test_cholesky_qr_matches_householder(),
    "Rayleigh-Ritz": lambda f: TC.test_rayleigh_ritz(f["tiny"]),
    "FD rationals": lambda f: TH.test_fd_exact_rationals(),
    "FD symbol order": lambda f: TH.test_fd_symbol_order(),
    "Kronecker sum on a box": lambda f: TH.test_laplacian_is_kronecker_sum_on_box(),
    "plane wave": lambda f: TH.test_laplacian_plane_wave_interior(),
    "Dirichlet box spectrum": lambda f: TH.test_dirichlet_box_spectrum(),
    "V_loc closed form": lambda f: TH.test_local_potential_closed_form(),
    "projector normalisation": lambda f: TH.test_projectors_normalised_and_orthogonal(),
    "apply = dense": lambda f: TH.test_apply_matches_dense(),
    "Hilbert bijection, unit steps": lambda f: TG.test_hilbert_bijection_and_unit_steps(3),
    "Hilbert order 1 = Gray walk": lambda f: TG.test_hilbert_order1_is_gray_walk(),
    "Hilbert bits minimal": lambda f: TG.test_hilbert_bits_is_the_smallest_cube_holding_the_blocks(),
    "sphere points brute force": lambda f: TG.test_sphere_points_brute_force(3.5, 0.7),
    "sums of three squares": lambda f: TG.test_sphere_point_counts_are_sums_of_three_squares(),
    "neighbours brute force": lambda f: TG.test_neighbour_table_brute_force(),
    "offset order": lambda f: TG.test_offsets_order(),
    "LDA potential = derivative": lambda f: TS.test_lda_potential_is_derivative(),
    "PZ81 slope continuity": lambda f: TS.test_lda_correlation_slope_continuous_at_rs_1(),
    "Anderson on a linear fixed point": lambda f: TS.test_anderson_solves_linear_fixed_point(),
    "Harris-Foulkes = Kohn-Sham": lambda f: TS.test_harris_foulkes_equals_kohn_sham_at_self_consistency(f["sih4"]),
    "density charge and invariance": lambda f: TS.test_density_counts_two_electrons_per_occupied_state(),
    "ion-ion pairs": lambda f: TS.test_ion_energy_pair(),
    "SRE closed forms": lambda f: TS.test_sre_is_density_weighted_rms_of_the_potential_change_in_rydberg(),
    "conv brute force": lambda f: TU.test_conv_matches_brute_force(3, 1),
    "SiLU gradient": lambda f: TU.test_silu_grad(),
    "Adam first step": lambda f: TU.test_adam_first_step_is_signed_lr(),
    "MSE closed forms": lambda f: TU.test_mse_is_the_mean_square_and_its_gradient(),
    "upsample adjoint": lambda f: TU.test_upsample_adjoint(),
    "point-wise H X = grid operator": lambda f: TH.test_pointwise_apply_matches_grid_operator(),
    "Hilbert block layout": lambda f: TG.test_ordering_layout(G.ORDER_HILBERT),
    "LDA derivative, both branches": lambda f: TS.test_lda_energy_derivative_on_both_branches(),
    "SAD normalisation": lambda f: TS.test_sad_density_normalised(),
    "SAD profile per species": lambda f: TS.test_sad_density_profile_per_species(),
    "addition theorem": lambda f: TS.test_solid_harmonics_addition_theorem(),
    "multipole exterior": lambda f: TS.test_multipole_potential_exterior(),
    "ghost points brute force": lambda f: TS.test_ghost_points_brute_force(),
    "CG = dense solve": lambda f: TS.test_conjugate_gradient_matches_dense_solve(),
    "Poisson: Gaussian charge": lambda f: TS.test_poisson_gaussian_charge((0.9, -0.6, 0.5)),
    "conv backward finite differences": lambda f: TU.test_conv_backward_finite_differences(1),
    "high-pass closed forms": lambda f: TU.test_gaussian_highpass_closed_forms(),
}

# slip -> (object patched, attribute, wrong version, pins that cover it)
CASES = {
    "filter beta_k squared": (C, "filter_scalars", filter_scalars_beta_squared,
                              ["filter = polynomial on eigenpairs", "filter scalars = Chebyshev ratios"]),
    "filter sigma_1 sign": (C, "filter_scalars", filter_scalars_sigma1_sign,
                            ["filter = polynomial on eigenpairs", "filter scalars = Chebyshev ratios"]),
    "filter drops the shift c": (C, "chebyshev_filter", filter_without_shift,
                                 ["filter = polynomial on eigenpairs", "filter normalisation"]),
    "filter applies H to Y_{k-2}": (C, "chebyshev_filter", filter_h_on_older_iterate,
                                    ["filter = polynomial on eigenpairs", "filter normalisation"]),
    "Lanczos bound without residual": (C, "lanczos_bound", lanczos_without_residual, ["Lanczos upper bound"]),
    "Cholesky lower factor as R": (C, "cholesky_qr", cholesky_qr_lower_factor, ["Cholesky-QR = Householder"]),
    "Ritz rotation transposed": (C, "rayleigh_ritz", rayleigh_ritz_rotation_transposed, ["Rayleigh-Ritz"]),
    "Rayleigh-Ritz without H": (C, "rayleigh_ritz", rayleigh_ritz_without_h, ["Rayleigh-Ritz"]),
    "FD weight sign": (OH, "fd_coefficients_exact", fd_weights_sign, ["FD rationals", "FD symbol order"]),
    "Laplacian centre weight once": (OH, "laplacian", laplacian_centre_once,
                                     ["Kronecker sum on a box", "plane wave", "Dirichlet box spectrum"]),
    "Laplacian over h, not h^2": (OH, "laplacian", laplacian_over_h,
                                  ["Kronecker sum on a box", "plane wave", "Dirichlet box spectrum"]),
    "Laplacian signed weight index": (OH, "laplacian", laplacian_signed_index,
                                      ["Kronecker sum on a box", "plane wave"]),
    "V_loc limit without 2": (OH, "local_potential", vloc_limit_without_2, ["V_loc closed form"]),
    "V_loc erf argument": (OH, "local_potential", vloc_erf_argument, ["V_loc closed form"]),
    "p projector normalisation": (OH, "projector_matrix", projectors_p_norm, ["projector normalisation"]),
    "KB term without h^3": (OH.Hamiltonian, "apply", apply_kb_without_h3, ["apply = dense"]),
    "kinetic sign": (OH.Hamiltonian, "apply", apply_kinetic_sign, ["apply = dense"]),
    "Hilbert without Gray encoding": (G, "hilbert_index3", hilbert_without_gray_decode,
                                      ["Hilbert bijection, unit steps", "Hilbert order 1 = Gray walk"]),
    "Hilbert bits z first": (G, "hilbert_index3", hilbert_z_first,
                             ["Hilbert bijection, unit steps", "Hilbert order 1 = Gray walk"]),
    "Hilbert bits of n": (G, "hilbert_bits", hilbert_bits_of_count, ["Hilbert bits minimal"]),
    "sphere boundary dropped": (G, "sphere_points", sphere_points_strict,
                                ["sphere points brute force", "sums of three squares"]),
    "neighbour offset sign": (G, "neighbour_table", neighbour_table_sign, ["neighbours brute force"]),
    "offsets +k before -k": (G, "offsets", offsets_positive_first, ["offset order"]),
    "LDA potential sign": (S, "lda", lda_potential_sign, ["LDA potential = derivative"]),
    "PZ81 B coefficient sign": (S, "PZ_B", 0.048, ["LDA potential = derivative"]),
    "PZ81 A coefficient mistyped": (S, "PZ_A", 0.0331, ["LDA potential = derivative", "PZ81 slope continuity"]),
    "PZ81 C coefficient sign": (S, "PZ_C", -0.0020, ["LDA potential = derivative", "PZ81 slope continuity"]),
    "Anderson extrapolation sign": (S.Anderson, "mix", anderson_extrapolation_sign,
                                    ["Anderson on a linear fixed point"]),
    "Harris-Foulkes full Hartree": (S, "harris_foulkes", _harris_foulkes(2.0, 1.0, 1.0),
                                    ["Harris-Foulkes = Kohn-Sham"]),
    "Harris-Foulkes single occupation": (S, "harris_foulkes", _harris_foulkes(1.0, 0.5, 1.0),
                                         ["Harris-Foulkes = Kohn-Sham"]),
    "Harris-Foulkes without xc double counting": (S, "harris_foulkes", _harris_foulkes(2.0, 0.5, 0.0),
                                                  ["Harris-Foulkes = Kohn-Sham"]),
    "density single occupation": (S, "density", density_single_occupation, ["density charge and invariance"]),
    "density without h^3": (S, "density", density_without_h3, ["density charge and invariance"]),
    "ion-ion pairs twice": (S, "ion_energy", ion_energy_all_ordered_pairs, ["ion-ion pairs"]),
    "SRE in Hartree": (S, "sre_ry", sre_in_hartree, ["SRE closed forms"]),
    "SRE without the root": (S, "sre_ry", sre_without_root, ["SRE closed forms"]),
    "conv kernel flipped": (U, "conv3d", conv_flipped_kernel, ["conv brute force"]),
    "SiLU gradient first term": (U, "silu_grad", silu_grad_first_term_only, ["SiLU gradient"]),
    "MSE summed": (U, "mse", mse_sum, ["MSE closed forms"]),
    "Adam without bias correction": (U, "adam_step", adam_without_bias_correction, ["Adam first step"]),
    "upsample backward mean": (U, "upsample_backward", upsample_backward_mean, ["upsample adjoint"]),
    "point-wise H X drops the KB term": (OH, "apply_at_points", pointwise_without_kb,
                                         ["point-wise H X = grid operator"]),
    "block-local index y fastest": (G, "build_grid", build_grid_local_xy_swapped, ["Hilbert block layout"]),
    "LDA derivative branch": (S, "lda_deps_drs", lda_derivative_branch, ["LDA derivative, both branches"]),
    "SAD normalisation without h^3": (S, "sad_density", sad_density_unnormalised, ["SAD normalisation"]),
    "SAD widths swapped between species": (S, "sad_density", sad_density_widths_swapped,
                                           ["SAD profile per species"]),
    "SAD Gaussian exponent halved": (S, "sad_density", sad_density_half_exponent, ["SAD profile per species"]),
    "SAD normalisation power of alpha": (S, "sad_density", sad_density_norm_power_one, ["SAD profile per species"]),
    "SAD Si charge 1": (S, "sad_density", sad_density_equal_charges, ["SAD profile per species"]),
    "solid harmonic l=2 scale": (S, "solid_harmonics", solid_harmonics_unscaled_l2,
                                 ["addition theorem", "multipole exterior"]),
    "multipole moments without h^3": (S, "multipole_moments", multipole_moments_without_h3,
                                      ["multipole exterior"]),
    "multipole exponent": (S, "multipole_potential", multipole_potential_exponent, ["multipole exterior"]),
    "ghost points signed weight index": (S, "ghost_points", ghost_points_signed_k, ["ghost points brute force"]),
    "CG beta inverted": (S, "conjugate_gradient", cg_beta_inverted, ["CG = dense solve"]),
    "Poisson source without 4 pi": (S, "hartree", hartree_source_without_4pi, ["Poisson: Gaussian charge"]),
    "Poisson boundary sign": (S, "hartree", hartree_boundary_sign, ["Poisson: Gaussian charge"]),
    "conv dW tap mirrored": (U, "conv3d_backward", conv_backward_dw_shift, ["conv backward finite differences"]),
    "high-pass weights unnormalised": (U, "gaussian_highpass", highpass_unnormalised, ["high-pass closed forms"]),
}


@pytest.fixture(scope="module")
def systems():
    return {"tiny": oracle_systems.tiny(), "sih4": oracle_systems.sih4_scf()}


def _fails(pin, systems) -> bool:
    try:
        pin(systems)
    except AssertionError:
        return True
    return False


def test_every_pin_passes_on_the_oracle_as_written(systems):
    failing = [name for name, pin in PINS.items() if _fails(pin, systems)]
    assert not failing, failing


@pytest.mark.parametrize("slip", sorted(CASES))
def test_planted_slip_fails_a_pin(slip, systems, monkeypatch):
    target, attr, wrong, pins = CASES[slip]
    monkeypatch.setattr(target, attr, wrong)
    caught = [p for p in pins if _fails(PINS[p], systems)]
    assert caught, f"no pin catches the slip '{slip}'"
