"""Pins of the oracle's SCF pieces: multipole harmonics against the Legendre
addition theorem, the Poisson solver against the analytic potential of
Gaussian charges, LDA potentials against numerical derivatives of the
energy density, Anderson mixing on a linear fixed point, and a small SCF
whose converged eigenvalues are those of its own final Hamiltonian."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import erf, eval_legendre

from oracle import grid as G
from oracle import hamiltonian as OH
from oracle import scf as S
from synth.cluster import random_block

import oracle_systems
from oracle_systems import H_POS


def test_solid_harmonics_addition_theorem():
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal((2, 3, 50))
    Ra = S.solid_harmonics(*a)
    Rb = S.solid_harmonics(*b)
    na = np.sqrt((a ** 2).sum(0))
    nb = np.sqrt((b ** 2).sum(0))
    cosg = (a * b).sum(0) / (na * nb)
    for l in range(5):
        sel = S.SH_L == l
        lhs = (Ra[sel] * Rb[sel]).sum(0)
        rhs = na ** l * nb ** l * eval_legendre(l, cosg)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def _gauss(g, centre, s, q):
    d2 = ((g.xyz - centre) ** 2).sum(1)
    return q * (2 * math.pi * s * s) ** -1.5 * np.exp(-d2 / (2 * s * s))


@pytest.mark.parametrize("centre", [(0.0, 0.0, 0.0), (0.9, -0.6, 0.5)])
def test_poisson_gaussian_charge(centre):
    g = G.build_grid(9.0, 0.45)
    nbr = G.neighbour_table(g)
    lap = OH.laplacian(g, nbr)
    s, q = 1.1, 2.0
    rho = _gauss(g, np.array(centre), s, q)
    v, it = S.hartree(g, lap, nbr, rho)
    d = np.sqrt(((g.xyz - np.array(centre)) ** 2).sum(1))
    exact = q * erf(d / (math.sqrt(2) * s)) / np.where(d > 0, d, 1)
    exact = np.where(d > 0, exact, q * math.sqrt(2 / math.pi) / s)
    assert np.abs(v - exact).max() < 2e-4 * exact.max()
    # the discrete residual of the solve is tiny by construction
    assert it > 10


def test_multipole_potential_exterior():
    g = G.build_grid(7.0, 0.4)
    c = np.array([0.8, 0.3, -0.5])
    rho = _gauss(g, c, 0.7, 1.5)
    q = S.multipole_moments(g, rho)
    pts = np.array([[9.0, 0.0, 0.0], [0.0, -8.5, 3.0], [5.0, 5.0, 5.0]])
    v = S.multipole_potential(q, pts)
    exact = 1.5 / np.sqrt(((pts - c) ** 2).sum(1))
    assert np.allclose(v, exact, rtol=5e-5)


def test_lda_potential_is_derivative():
    rho = np.array([1e-4, 3e-3, 0.02, 0.07, 0.2, 0.5, 2.0])
    eps, v = S.lda(rho)
    d = 1e-6 * rho
    ep, _ = S.lda(rho + d)
    em, _ = S.lda(rho - d)
    num = ((rho + d) * ep - (rho - d) * em) / (2 * d)
    assert np.allclose(v, num, rtol=1e-7)
    # exchange part: -(3/4)(3 rho / pi)^(1/3)
    rs = (3 / (4 * math.pi * rho)) ** (1 / 3)
    ex = -0.75 * (3 * rho / math.pi) ** (1 / 3)
    assert np.allclose(eps - S.lda_eps(rs) + (-S.EX_CONST / rs) - ex, 0.0, atol=1e-14)
    # the two correlation branches nearly meet at r_s = 1
    lo = S.PZ_A * 0 + S.PZ_B + 0 + S.PZ_D
    hi = S.PZ_GAMMA / (1 + S.PZ_BETA1 + S.PZ_BETA2)
    assert abs(lo - hi) < 2e-4
    assert np.all(S.lda(np.array([0.0, 1e-15, -1e-3]))[1] == 0.0)


def test_lda_energy_derivative_on_both_branches():
    # d eps / d r_s against central differences of eps, on each side of r_s = 1
    rs = np.array([0.05, 0.3, 0.9, 0.999, 1.001, 1.5, 4.0, 20.0])
    d = 1e-6 * rs
    num = (S.lda_eps(rs + d) - S.lda_eps(rs - d)) / (2 * d)
    assert np.allclose(S.lda_deps_drs(rs), num, rtol=1e-7)


def test_lda_correlation_slope_continuous_at_rs_1():
    # the PZ81 fit joins its two correlation forms at r_s = 1 with matching value and slope;
    # the slope brings in the coefficients A and C, which vanish from the value there
    d = 1e-9
    lo, hi = S.lda_deps_drs(np.array([1.0 - d, 1.0 + d]))
    assert abs(lo - hi) < 1e-4
    assert abs(hi - S.lda_deps_drs(np.array([1.0 + 1e-3]))[0]) < 1e-3


def test_conjugate_gradient_matches_dense_solve():
    rng = np.random.default_rng(4)
    n = 40
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    b = rng.standard_normal(n)
    x, it = S.conjugate_gradient(lambda v: A @ v, b, np.zeros(n), rtol=1e-13)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-11 * np.abs(x).max())
    assert 0 < it <= 2 * n
    # a start at the solution needs no iteration
    x2, it2 = S.conjugate_gradient(lambda v: A @ v, b, np.linalg.solve(A, b), rtol=1e-10)
    assert it2 == 0


def test_ghost_points_brute_force():
    # each (inside point, stencil offset) whose target lies outside the sphere, by plain loops
    g = G.build_grid(3.2, 0.8)
    nbr = G.neighbour_table(g)
    owner, k, pts = S.ghost_points(g, nbr)
    thr = math.floor((g.radius / g.h) ** 2 + 1e-9)
    want = []
    for r, (i, j, l) in enumerate(g.ijk.tolist()):
        for axis in range(3):
            for s in list(range(-6, 0)) + list(range(1, 7)):
                q = [i, j, l]
                q[axis] += s
                if q[0] ** 2 + q[1] ** 2 + q[2] ** 2 > thr:
                    want.append((r, abs(s), q[0], q[1], q[2]))
    got = [(int(o), int(kk), *np.rint(p / g.h).astype(int).tolist()) for o, kk, p in zip(owner, k, pts)]
    assert sorted(got) == sorted(want)
    assert np.allclose(pts / g.h, np.rint(pts / g.h), atol=1e-12)


def test_anderson_solves_linear_fixed_point():
    rng = np.random.default_rng(1)
    n = 5
    A = rng.standard_normal((n, n))
    A = 0.3 * A / np.linalg.norm(A, 2)
    c = rng.standard_normal(n)
    x_star = np.linalg.solve(np.eye(n) - A, c)
    mix = S.Anderson(beta=0.3, history=6)
    x = np.zeros(n)
    for _ in range(8):
        x = mix.mix(x, A @ x + c - x)
    assert np.allclose(x, x_star, atol=1e-10)


def test_ion_energy_pair():
    pos = np.array([[0.0, 0.0, 0.0], [0.0, 3.0, 4.0], [1.0, 0.0, 0.0]])
    z = np.array([4.0, 1.0, 1.0])
    expect = 4 / 5 + 4 / 1 + 1 / math.sqrt(1 + 9 + 16)
    assert abs(S.ion_energy(pos, z) - expect) < 1e-14


def test_sad_density_normalised():
    g = G.build_grid(9.0, 0.7)
    rho = S.sad_density(g, np.array([[0.0, 0, 0], [2.8, 0, 0]]), np.array([0, 1], np.int32), 5)
    assert abs(g.h ** 3 * rho.sum() - 5) < 1e-12 and (rho > 0).all()


def test_sad_density_profile_per_species():
    # A normalised Gaussian (alpha / pi)^(3/2) exp(-alpha r^2) carries unit
    # charge and has <r^2> = 3 / (2 alpha).  One Si and one H, 36.4 bohr apart
    # and 21 bohr from the wall, each sitting on a grid point: the charge on
    # each side of the midplane is that species' Z, and its second moment
    # about its own atom is Z * 3 / (2 alpha) for that species' alpha.  The
    # grid sums of these smooth Gaussians are exact far below 1e-9.
    h, a_si, a_h = 0.7, 0.074, 0.21
    g = G.build_grid(39.2, h)
    pos = np.array([[-18.2, 0.0, 0.0], [18.2, 0.0, 0.0]])
    rho = S.sad_density(g, pos, np.array([0, 1], np.int32), 5, alpha_si=a_si, alpha_h=a_h)
    left = g.xyz[:, 0] < 0
    h3 = h ** 3
    for side, z, alpha, centre in ((left, 4.0, a_si, pos[0]), (~left, 1.0, a_h, pos[1])):
        q = h3 * rho[side].sum()
        m2 = h3 * (rho[side] * ((g.xyz[side] - centre) ** 2).sum(axis=1)).sum()
        assert abs(q - z) < 1e-9 * z, (q, z)
        assert abs(m2 - 1.5 * z / alpha) < 1e-9 * (1.5 * z / alpha), (m2, 1.5 * z / alpha)


def test_density_counts_two_electrons_per_occupied_state():
    # with orthonormal columns X the orbitals X_i / h^(3/2) are normalised in
    # the grid quadrature, and each occupied state holds two electrons:
    # h^3 sum rho = 2 n_occ.  The density is the diagonal of the projector on
    # the occupied span, so a rotation inside the occupied columns and any
    # change of the other columns leave it unchanged.
    h = 0.7
    X, _ = np.linalg.qr(np.random.default_rng(8).standard_normal((500, 12)))
    for n_occ in (1, 5, 12):
        rho = S.density(X, n_occ, h)
        assert abs(h ** 3 * rho.sum() - 2 * n_occ) < 1e-12 and (rho >= 0).all()
    U, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((5, 5)))
    Y = X.copy()
    Y[:, :5] = X[:, :5] @ U
    Y[:, 5:] = np.random.default_rng(10).standard_normal((500, 7))
    ref = S.density(X, 5, h)
    assert np.allclose(S.density(Y, 5, h), ref, rtol=0, atol=1e-13 * ref.max())


def test_sre_is_density_weighted_rms_of_the_potential_change_in_rydberg():
    # SRE = sqrt(int rho dV^2 / N_e) in Hartree, reported in Rydberg (1 Ha = 2 Ry)
    g = G.build_grid(6.0, 0.7)
    rho = S.sad_density(g, np.zeros((1, 3)), np.array([0], np.int32), 4)     # 4 electrons
    # a uniform change of delta Ha everywhere: SRE = |delta| Ha = 2 |delta| Ry
    assert abs(S.sre_ry(g.h, rho, np.full(g.n, 3e-3), 4) - 6e-3) < 1e-15
    assert S.sre_ry(g.h, rho, np.zeros(g.n), 4) == 0.0
    # a fraction f of the charge sees d1, the rest d2: the root of the weighted mean square
    inner = (g.xyz ** 2).sum(1) < 9.0
    f = g.h ** 3 * rho[inner].sum() / 4
    assert 0.1 < f < 0.9
    dv = np.where(inner, 0.01, -0.002)
    assert abs(S.sre_ry(g.h, rho, dv, 4) - 2 * math.sqrt(f * 0.01 ** 2 + (1 - f) * 0.002 ** 2)) < 1e-15


@pytest.fixture(scope="module")
def sih4_scf():
    return oracle_systems.sih4_scf()


def test_scf_converges_and_is_self_consistent(sih4_scf):
    H, nbr, st, reps = sih4_scf
    assert reps[-1].sre_ry < 1e-4
    assert reps[0].sre_ry > 1e-2
    # the tracked eigenvalues are those of the final Hamiltonian (V built from rho_in)
    lam = np.linalg.eigvalsh(H.dense())
    assert np.allclose(reps[-1].eig[:4], lam[:4], atol=1e-8)
    assert reps[-1].lumo - reps[-1].homo > 0.05
    # Harris-Foulkes energy settles
    assert abs(reps[-1].energy - reps[-2].energy) < 1e-7


def test_scf_energy_stationary(sih4_scf):
    # near self-consistency the Harris-Foulkes functional is stationary: the
    # SRE-weighted change of energy is second order
    _, _, _, reps = sih4_scf
    e = np.array([r.energy for r in reps])
    sre = np.array([r.sre_ry for r in reps])
    late = slice(10, None)
    assert np.all(np.abs(e[late] - e[-1]) < 10 * sre[late] ** 2 + 1e-8)


def test_harris_foulkes_equals_kohn_sham_at_self_consistency(sih4_scf):
    """The Harris-Foulkes energy at the input density equals the Kohn-Sham
    functional evaluated directly at the output density up to second order in
    their difference: kinetic + local + nonlocal from the orbitals, Hartree as
    half the Coulomb self-energy, LDA exchange-correlation, ion-ion."""
    H, nbr, st, reps = sih4_scf
    g = H.grid
    h3 = g.h ** 3
    n_occ = 4
    e_ii = S.ion_energy(np.array(H_POS), OH.PseudoParams().charges(np.array([0, 1, 1, 1, 1], np.int32)))
    rho_in = st.rho_in
    vh_in, _ = S.hartree(g, H.lap, nbr, rho_in)
    exc_in, vxc_in = S.lda(rho_in)
    Hin = dataclasses.replace(H, veff=H.vloc + vh_in + vxc_in)
    lam, V = np.linalg.eigh(Hin.dense())
    psi = V[:, :n_occ] / math.sqrt(h3)              # normalised in h^3 sum psi^2 = 1
    e_hf = S.harris_foulkes(g.h, lam, n_occ, rho_in, vh_in, exc_in, vxc_in, e_ii)
    # direct functional at the output density
    rho_out = 2.0 * (psi ** 2).sum(1)
    Hext = dataclasses.replace(H, veff=H.vloc)
    e_one = 2.0 * h3 * float((psi * Hext.apply(psi)).sum())
    vh_out, _ = S.hartree(g, H.lap, nbr, rho_out)
    exc_out, _ = S.lda(rho_out)
    e_ks = e_one + 0.5 * h3 * float(rho_out @ vh_out) + h3 * float(rho_out @ exc_out) + e_ii
    drho = math.sqrt(h3 * float(((rho_out - rho_in) ** 2).sum()))
    assert drho < 1e-3
    assert abs(e_hf - e_ks) < 1e-6
    # far from self-consistency (the superposed atomic start) the two differ clearly
    rho0 = S.sad_density(g, np.array(H_POS), np.array([0, 1, 1, 1, 1], np.int32), 8)
    vh0, _ = S.hartree(g, H.lap, nbr, rho0)
    exc0, vxc0 = S.lda(rho0)
    lam0, V0 = np.linalg.eigh(dataclasses.replace(H, veff=H.vloc + vh0 + vxc0).dense())
    psi0 = V0[:, :n_occ] / math.sqrt(h3)
    r0 = 2.0 * (psi0 ** 2).sum(1)
    vh0o, _ = S.hartree(g, H.lap, nbr, r0)
    e_ks0 = (2.0 * h3 * float((psi0 * Hext.apply(psi0)).sum()) + 0.5 * h3 * float(r0 @ vh0o)
             + h3 * float(r0 @ S.lda(r0)[0]) + e_ii)
    e_hf0 = S.harris_foulkes(g.h, lam0, n_occ, rho0, vh0, exc0, vxc0, e_ii)
    assert abs(e_hf0 - e_ks0) > 100 * abs(e_hf - e_ks)


def test_resume_from_saved_state_is_bit_exact(tmp_path):
    """What an SCF carries between steps (rho_in, V_H warm start, X, filter
    bounds, step counter, Anderson history) saved to .npz and loaded into a
    fresh state reproduces the next step exactly."""
    pos = np.array(H_POS)
    species = np.array([0, 1, 1, 1, 1], np.int32)
    g = G.build_grid(float(np.sqrt((pos ** 2).sum(1)).max()) + 5.0, 0.7)
    nbr = G.neighbour_table(g)
    pp = OH.PseudoParams()
    H = OH.build_hamiltonian(g, pos, species, pp)
    eii = S.ion_energy(pos, pp.charges(species))
    v0 = random_block(g.n, 1, 6)[:, 0]
    st = S.ScfState(S.sad_density(g, pos, species, 8), random_block(g.n, 10, 5), np.zeros(g.n))
    for _ in range(3):
        S.scf_step(H, nbr, st, 8, 12, v0, eii)
    f = tmp_path / "state.npz"
    np.savez(f, rho_in=st.rho_in, X=st.X, vh=st.vh, a=st.a, a0=st.a0, step=st.step,
             beta=st.mixer.beta, history=st.mixer.history, xs=np.array(st.mixer.xs), fs=np.array(st.mixer.fs))
    z = np.load(f)
    mixer = S.Anderson(float(z["beta"]), int(z["history"]))
    mixer.xs, mixer.fs = [x.copy() for x in z["xs"]], [x.copy() for x in z["fs"]]
    resumed = S.ScfState(z["rho_in"].copy(), z["X"].copy(), z["vh"].copy(), float(z["a"]), float(z["a0"]),
                         int(z["step"]), mixer)
    r1 = S.scf_step(H, nbr, st, 8, 12, v0, eii)
    r2 = S.scf_step(H, nbr, resumed, 8, 12, v0, eii)
    assert r1.step == r2.step == 4
    assert r1.energy == r2.energy and r1.sre_ry == r2.sre_ry
    assert np.array_equal(r1.eig, r2.eig)
    assert np.array_equal(st.rho_in, resumed.rho_in) and np.array_equal(st.X, resumed.X)
