"""Oracle: Chebyshev-filtered subspace iteration (ChFSI) pieces.

Paper: instead of computing individual eigenpairs, ChFSI improves an
invariant subspace of the lowest states together with the potentials over
the SCF iterations (the CheFSI paragraph); its efficiency rests on sparse
H-times-vector products.  The paper defers the algorithm itself to the PARSEC
ChFSI reference; the steps below are the standard Zhou-Saad form:

* filter: Y = T_m((H - c) / e) X / T_m((a0 - c) / e), e = (b - a) / 2,
  c = (b + a) / 2, evaluated by the Chebyshev three-term recurrence with the
  scaling folded in (sigma_k = T_{k-1}(t0) / T_k(t0), t0 = (a0 - c) / e);
* b from a k-step Lanczos run (largest Ritz value plus the residual norm);
* Cholesky-QR: S = X^T X = R^T R, X <- X R^{-1};
* Rayleigh-Ritz: Hs = X^T (H X) symmetrised, Hs = Q diag(lambda) Q^T,
  X <- X Q, eigenvalues ascending.
"""
from __future__ import annotations

import numpy as np


def filter_scalars(m: int, a: float, b: float, a0: float) -> list[tuple[float, float, float]]:
    """Per degree step k = 1..m the coefficients (alpha_k, c, beta_k) with
    Y_k = alpha_k (H Y_{k-1} - c Y_{k-1}) - beta_k Y_{k-2}  (beta_1 = 0)."""
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma1 = e / (a0 - c)
    out = [(sigma1 / e, c, 0.0)]
    sigma = sigma1
    for _ in range(2, m + 1):
        sigma_next = 1.0 / (2.0 / sigma1 - sigma)
        out.append((2.0 * sigma_next / e, c, sigma * sigma_next))
        sigma = sigma_next
    return out


def chebyshev_filter(apply_h, X: np.ndarray, m: int, a: float, b: float, a0: float) -> np.ndarray:
    """Scaled degree-m Chebyshev filter of X (damps [a, b], normalised at a0)."""
    prev = X
    cur = X
    for k, (alpha, c, beta) in enumerate(filter_scalars(m, a, b, a0)):
        hx = apply_h(cur)
        nxt = alpha * (hx - c * cur)
        if k > 0:
            nxt = nxt - beta * prev
        prev, cur = cur, nxt
    return cur


def lanczos_bound(apply_h, v0: np.ndarray, k: int = 10) -> tuple[float, float, float]:
    """k-step Lanczos on v0 (no reorthogonalisation).

    Returns (upper bound b = theta_max + ||f_k||, theta_min, theta_max)."""
    v = v0 / np.linalg.norm(v0)
    f = apply_h(v)
    alpha = float(v @ f)
    f = f - alpha * v
    T = np.zeros((k, k))
    T[0, 0] = alpha
    for j in range(1, k):
        beta = float(np.linalg.norm(f))
        v_prev, v = v, f / beta
        f = apply_h(v) - beta * v_prev
        alpha = float(v @ f)
        f = f - alpha * v
        T[j, j] = alpha
        T[j, j - 1] = T[j - 1, j] = beta
    theta = np.linalg.eigvalsh(T)
    return float(theta[-1] + np.linalg.norm(f)), float(theta[0]), float(theta[-1])


def cholesky_qr(X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Q = X R^{-1} with S = X^T X = R^T R (R upper, positive diagonal)."""
    S = X.T @ X
    R = np.linalg.cholesky(S).T
    Q = np.linalg.solve(R.T, X.T).T
    return Q, R


def rayleigh_ritz(apply_h, X: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Ritz values (ascending) and rotated vectors X Q of an orthonormal X."""
    W = apply_h(X)
    Hs = X.T @ W
    Hs = 0.5 * (Hs + Hs.T)
    lam, Q = np.linalg.eigh(Hs)
    return lam, X @ Q


def chfsi_iteration(apply_h, X: np.ndarray, m: int, a: float, b: float, a0: float):
    """One ChFSI iteration: filter, Cholesky-QR, Rayleigh-Ritz."""
    Y = chebyshev_filter(apply_h, X, m, a, b, a0)
    Q, _ = cholesky_qr(Y)
    lam, Xn = rayleigh_ritz(apply_h, Q)
    return lam, Xn
