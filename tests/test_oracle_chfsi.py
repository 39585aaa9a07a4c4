"""Pins of the oracle's ChFSI pieces against dense linear algebra on tiny
grids: the filter against the Chebyshev polynomial evaluated on the exact
eigenpairs, Lanczos against the exact spectrum, Cholesky-QR against
Householder QR, Rayleigh-Ritz against eigh, and the full iteration against
the exact lowest eigenvalues."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import chfsi as C

import oracle_systems


@pytest.fixture(scope="module")
def tiny():
    return oracle_systems.tiny()


def test_filter_equals_polynomial_on_eigenpairs(tiny):
    H, Hd, lam, V = tiny
    X = np.random.default_rng(0).standard_normal((Hd.shape[0], 6))
    a, b, a0 = lam[40], lam[-1] * 1.01, lam[0]
    for m in (1, 2, 5, 10):
        Y = C.chebyshev_filter(H.apply, X, m, a, b, a0)
        e, c = (b - a) / 2, (b + a) / 2
        coef = np.zeros(m + 1)
        coef[m] = 1.0
        p = npcheb.chebval((lam - c) / e, coef) / npcheb.chebval((a0 - c) / e, coef)
        expect = V @ (p[:, None] * (V.T @ X))
        assert np.allclose(Y, expect, rtol=0, atol=1e-9 * np.abs(expect).max())


def test_filter_scalars_normalisation():
    # the scaled polynomial is 1 at a0 and bounded by 1 / |T_m(t0)| on [a, b]
    a, b, a0, m = -0.2, 3.0, -1.0, 8

    def scalar_h(x):
        return lam_pt * x

    for lam_pt, bound in ((a0, None), (a, True), (b, True), (0.5 * (a + b), True)):
        y = C.chebyshev_filter(scalar_h, np.array([1.0]), m, a, b, a0)[0]
        t0 = (a0 - (a + b) / 2) / ((b - a) / 2)
        tm = np.cosh(m * np.arccosh(abs(t0)))
        if bound is None:
            assert abs(y - 1.0) < 1e-13
        else:
            assert abs(y) <= 1.0 / tm * (1 + 1e-12)


def test_lanczos_upper_bound(tiny):
    H, Hd, lam, _ = tiny
    v0 = np.random.default_rng(3).standard_normal(Hd.shape[0])
    b, tmin, tmax = C.lanczos_bound(H.apply, v0, 10)
    assert b >= lam[-1] - 1e-10
    assert b < lam[-1] * 1.5
    assert tmin >= lam[0] - 1e-10 and tmax <= lam[-1] + 1e-10


def test_cholesky_qr_matches_householder():
    X = np.random.default_rng(4).standard_normal((300, 12))
    Q, R = C.cholesky_qr(X)
    Qh, Rh = np.linalg.qr(X)
    s = np.sign(np.diag(Rh))
    assert np.allclose(R, s[:, None] * Rh, atol=1e-11)
    assert np.allclose(Q, Qh * s[None, :], atol=1e-11)
    assert np.allclose(Q.T @ Q, np.eye(12), atol=1e-13)
    assert np.allclose(np.triu(R), R)


def test_rayleigh_ritz(tiny):
    H, Hd, lam, V = tiny
    n = Hd.shape[0]
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((n, 7)))
    ritz, Xr = C.rayleigh_ritz(H.apply, Q)
    assert np.allclose(ritz, np.linalg.eigvalsh(Q.T @ Hd @ Q), atol=1e-12)
    assert np.allclose(Xr.T @ Xr, np.eye(7), atol=1e-12)
    # Ritz condition: the rotated vectors diagonalise the projected operator,
    # column j carrying the j-th (ascending) Ritz value
    assert np.allclose(Xr.T @ Hd @ Xr, np.diag(ritz), atol=1e-10 * np.abs(ritz).max())
    U, _ = np.linalg.qr(np.random.default_rng(6).standard_normal((7, 7)))
    ritz2, _ = C.rayleigh_ritz(H.apply, Q @ U)
    assert np.allclose(ritz, ritz2, atol=1e-12)
    # the subspace of exact eigenvectors gives exact eigenvalues
    ritz3, _ = C.rayleigh_ritz(H.apply, V[:, 3:9])
    assert np.allclose(ritz3, lam[3:9], atol=1e-12)


def test_chfsi_converges_to_lowest_eigenvalues(tiny):
    H, Hd, lam, _ = tiny
    n, k = Hd.shape[0], 10
    X = np.random.default_rng(7).standard_normal((n, k))
    v0 = np.random.default_rng(8).standard_normal(n)
    b, tmin, _ = C.lanczos_bound(H.apply, v0)
    a0, a = tmin, tmin + 0.1 * (b - tmin)
    for _ in range(60):
        ritz, X = C.chfsi_iteration(H.apply, X, 12, a, b, a0)
        a, a0 = ritz[-1], ritz[0]
    # the lowest 8 of the 10 tracked values converge (the top two guard the gap)
    assert np.allclose(ritz[:8], lam[:8], atol=1e-10)


@pytest.mark.parametrize("m,a,b,a0", [(1, -0.2, 3.0, -1.0), (12, 0.1, 40.0, -0.5), (16, -2.0, 5.0, -2.3)])
def test_filter_scalars_are_chebyshev_ratios(m, a, b, a0):
    # dividing T_{k}(t) = 2 t T_{k-1}(t) - T_{k-2}(t) by T_k(t0), t = (x - c) / e, gives
    # alpha_k = 2 T_{k-1}(t0) / (e T_k(t0)) (alpha_1 = 1 / (e t0)) and beta_k = T_{k-2}(t0) / T_k(t0);
    # the T_k(t0) here come from numpy's Chebyshev series evaluation
    e, c = (b - a) / 2, (b + a) / 2
    t0 = (a0 - c) / e

    def T(k):
        coef = np.zeros(k + 1)
        coef[k] = 1.0
        return npcheb.chebval(t0, coef)

    got = C.filter_scalars(m, a, b, a0)
    assert len(got) == m
    for k, (alpha, cc, beta) in enumerate(got, start=1):
        assert cc == c
        assert alpha == pytest.approx(2 * T(k - 1) / (e * T(k)) if k > 1 else 1 / (e * t0), rel=1e-12)
        assert beta == (0.0 if k == 1 else pytest.approx(T(k - 2) / T(k), rel=1e-12))
