"""Pins of the oracle Hamiltonian: FD weights, operator assembly, potentials,
projectors, symmetry.  Each test compares against something the oracle does
not compute itself (exact rationals, Kronecker sums built from Toeplitz
matrices, analytic functions, continuum integrals)."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.special import erf

from oracle import grid as G
from oracle import hamiltonian as OH
from synth.cluster import make_cluster, random_block


def test_fd_exact_rationals():
    c = OH.fd_coefficients_exact()
    assert c == [Fraction(-5369, 1800), Fraction(12, 7), Fraction(-15, 56), Fraction(10, 189),
                 Fraction(-1, 112), Fraction(2, 1925), Fraction(-1, 16632)]
    assert OH.fd_coefficients_exact(1) == [Fraction(-2), Fraction(1)]


def test_fd_symbol_order():
    c = OH.fd_coefficients()
    for th in (0.05, 0.2, 0.4):
        sym = c[0] + 2 * sum(c[k] * math.cos(k * th) for k in range(1, 7))
        assert abs(sym + th * th) < 3 * th ** 14 + 1e-15
    sym_pi = c[0] + 2 * sum(c[k] * math.cos(k * math.pi) for k in range(1, 7))
    assert abs(sym_pi - (-7.07294)) < 1e-5


def _box_grid(n, h=0.6):
    """A Grid object whose points fill an n^3 cube (lex order) instead of a sphere."""
    g = np.arange(n)
    i, j, k = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([i.ravel(), j.ravel(), k.ravel()], 1)
    order = np.lexsort((pts[:, 0], pts[:, 1], pts[:, 2]))
    pts = pts[order] - n // 2
    return G.Grid(h, 0.0, n, pts, np.arange(len(pts)), len(pts), G.ORDER_LEX, np.zeros((0, 3), np.int64))


def test_laplacian_is_kronecker_sum_on_box():
    n, h = 9, 0.6
    g = _box_grid(n, h)
    L = OH.laplacian(g).toarray()
    c = OH.fd_coefficients()
    col = np.zeros(n)
    col[:7] = c
    T = sla.toeplitz(col) / h ** 2
    I = np.eye(n)
    # lex order with x fastest: index = x + n y + n^2 z
    K = np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)
    assert np.allclose(L, K, rtol=0, atol=1e-12)


def test_dirichlet_box_spectrum():
    """-1/2 L on an n^3 box with zero values outside: its spectrum is every sum of three
    eigenvalues of the 1-D stencil matrix, all of them inside the symbol's range
    [3 sigma(pi), 0] / h^2 (eigenvalues of a symmetric Toeplitz matrix lie in the range of
    its symbol), and the lowest one tends to the continuum box's 3 pi^2 / (2 ((n + 1) h)^2).
    With the wide stencil cut at the walls that limit is reached at first order: the
    relative error halves when n doubles."""
    from scipy.sparse.linalg import eigsh
    c = OH.fd_coefficients()
    sym_pi = c[0] + 2 * sum(c[k] * math.cos(k * math.pi) for k in range(1, 7))
    n, h = 7, 0.6
    lam = np.linalg.eigvalsh(OH.laplacian(_box_grid(n, h)).toarray())
    col = np.zeros(n)
    col[:7] = c
    t = np.linalg.eigvalsh(sla.toeplitz(col)) / h ** 2
    sums = np.sort((t[:, None, None] + t[None, :, None] + t[None, None, :]).ravel())
    assert np.allclose(lam, sums, rtol=0, atol=1e-11 * np.abs(sums).max())
    assert lam.max() < 0 and lam.min() > 3 * sym_pi / h ** 2
    errs = []
    for n in (9, 19, 39):
        low = eigsh(-0.5 * OH.laplacian(_box_grid(n, h)), k=1, which="SA")[0][0]
        exact = 3 * math.pi ** 2 / (2 * ((n + 1) * h) ** 2)
        errs.append(abs(low - exact) / exact)
    assert errs[2] < 0.012
    assert 1.6 < errs[0] / errs[1] < 2.4 and 1.6 < errs[1] / errs[2] < 2.4


def test_laplacian_plane_wave_interior():
    g = G.build_grid(8.0, 0.5)
    nbr = G.neighbour_table(g)
    L = OH.laplacian(g, nbr)
    k = np.array([0.7, -1.1, 0.4])
    f = np.cos(g.xyz @ k + 0.3)
    lf = L @ f
    c = OH.fd_coefficients()
    sym = sum(c[0] + 2 * sum(c[m] * math.cos(m * kk * g.h) for m in range(1, 7)) for kk in k) / g.h ** 2
    interior = (nbr >= 0).all(1)
    assert interior.sum() > 1000
    assert np.allclose(lf[interior], sym * f[interior], rtol=0, atol=1e-11)


def test_free_sphere_ground_state_converges():
    # -1/2 nabla^2 in a sphere with psi = 0 outside: lowest eigenvalue pi^2 / (2 R^2)
    from scipy.sparse.linalg import eigsh
    R = 3.0
    errs = []
    for h in (0.5, 0.3):
        g = G.build_grid(R, h)
        L = OH.laplacian(g)
        lam = eigsh(-0.5 * L, k=1, which="SA")[0][0]
        errs.append(abs(lam - math.pi ** 2 / (2 * R * R)) / (math.pi ** 2 / (2 * R * R)))
    assert errs[1] < errs[0] and errs[1] < 0.12


def _tiny_system():
    pos = np.array([[0.3, -0.2, 0.1], [2.6, 2.4, -2.5], [-1.4, 1.1, 1.5]])
    species = np.array([0, 0, 1], np.int32)
    g = G.build_grid(6.5, 0.7)
    return g, pos, species


def test_local_potential_closed_form():
    g, pos, species = _tiny_system()
    pp = OH.PseudoParams()
    v = OH.local_potential(g, pos, species, pp)
    rng = np.random.default_rng(0)
    for p in rng.choice(g.n, 20, replace=False):
        r = g.xyz[p]
        expect = 0.0
        for a in range(3):
            z = 4.0 if species[a] == 0 else 1.0
            w = pp.r_loc if species[a] == 0 else pp.r_loc_h
            d = math.dist(r, pos[a])
            expect -= z * math.erf(d / w) / d
        assert abs(v[p] - expect) < 1e-13 * abs(expect) + 1e-15
    # atom exactly on a grid point: the finite r -> 0 limit
    v0 = OH.local_potential(g, np.zeros((1, 3)), np.array([0], np.int32), pp)
    centre = np.nonzero((g.ijk == 0).all(1))[0][0]
    assert abs(v0[centre] + 2 * 4 / (math.sqrt(math.pi) * pp.r_loc)) < 1e-14
    d = 1e-4
    assert abs(v0[centre] + 4 * erf(d / pp.r_loc) / d) < 1e-6


def test_projectors_normalised_and_orthogonal():
    # continuum normalisation: h^3 sum beta^2 -> 1; s and p orthogonal on a grid
    # centred at the atom (parity of the grid)
    pp = OH.PseudoParams()
    g = G.build_grid(6.0, 0.35)
    B, e = OH.projector_matrix(g, np.zeros((1, 3)), np.array([0], np.int32), pp)
    Bd = B.toarray()
    gram = g.h ** 3 * Bd.T @ Bd
    assert np.allclose(np.diag(gram), 1.0, atol=2e-6)
    assert np.allclose(gram - np.diag(np.diag(gram)), 0.0, atol=1e-14)
    assert list(e) == [pp.h_s, pp.h_p, pp.h_p, pp.h_p]
    # the analytic s projector at the centre point
    centre = np.nonzero((g.ijk == 0).all(1))[0][0]
    assert abs(Bd[centre, 0] - math.sqrt(4 / (math.sqrt(math.pi) * pp.r_c ** 3)) / math.sqrt(4 * math.pi)) < 1e-15
    # the support is exactly the ball of radius r_cut
    d = np.sqrt((g.xyz ** 2).sum(1))
    assert np.array_equal(np.nonzero(Bd[:, 0])[0], np.nonzero(d <= pp.r_cut)[0])


# a nonzero p-channel energy so that every projector column is exercised
PP_TEST = OH.PseudoParams(h_s=2.0, h_p=0.5)


def test_hamiltonian_symmetric_and_rank():
    g, pos, species = _tiny_system()
    H = OH.build_hamiltonian(g, pos, species, PP_TEST)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, g.n))
    assert abs(x @ H.apply(y) - H.apply(x) @ y) < 1e-12 * abs(x @ H.apply(y))
    # nonlocal part: rank <= 4 per Si, positive semidefinite for positive energies
    Bd = H.B.toarray()
    nl = g.h ** 3 * (Bd * H.kb_energy) @ Bd.T
    w = np.linalg.eigvalsh(nl)
    assert (w > 1e-10).sum() == 8 and w.min() > -1e-12


def test_apply_matches_dense():
    g, pos, species = _tiny_system()
    H = OH.build_hamiltonian(g, pos, species, PP_TEST)
    X = np.random.default_rng(2).standard_normal((g.n, 5))
    assert np.allclose(H.apply(X), H.dense() @ X, rtol=0, atol=1e-11)


def test_pointwise_apply_matches_grid_operator():
    # the point-at-a-time evaluation (used for the full-size sampled parity)
    # against the assembled operator on a small grid, including points on
    # the sphere's surface and next to atoms
    c = make_cluster(4.8, 5)
    g = G.build_grid(c.domain_radius(), 0.9)
    H = OH.build_hamiltonian(g, c.pos, c.species, PP_TEST)
    X = random_block(g.n, 3, 1)
    Y = H.apply(X)
    key = {tuple(v): i for i, v in enumerate(g.ijk)}

    def x_at(pts):
        return np.array([X[key[tuple(p)]] for p in pts])

    r2 = (g.ijk ** 2).sum(axis=1)
    near_atom = np.argmin(((g.xyz[:, None, :] - c.pos[None, c.species == 0, :]) ** 2).sum(axis=2), axis=0)
    idx = np.concatenate([np.random.default_rng(0).choice(g.n, 12, replace=False), np.argsort(r2)[-6:], near_atom[:6]])
    ya, mag = OH.apply_at_points(g.ijk[idx], x_at, g.h, g.radius, c.pos, c.species, PP_TEST)
    assert np.abs(ya - Y[idx]).max() < 1e-12 * np.abs(Y).max()
    assert np.all(mag >= np.abs(ya) - 1e-12)
