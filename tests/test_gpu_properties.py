"""Properties that hold for any input: H is symmetric in the Euclidean inner
product of the grid rows (the stencil is symmetric, the KB term is B D B^T),
Ritz values do not depend on the basis of the subspace, and the error paths
report the documented codes (non-convergence, non-positive-definite Gram)."""
import numpy as np
import pytest

from synth.cluster import random_block
from gpu_system import build, to_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def system():
    return build()


@pytest.mark.parametrize("generic", [False, True])
def test_hamiltonian_is_symmetric(system, generic):
    s = system
    X = to_rows(s, random_block(s["g"].n, 8, 11), torch.float64)
    Yv = to_rows(s, random_block(s["g"].n, 8, 12), torch.float64)
    HX, HY = torch.empty_like(X), torch.empty_like(Yv)
    s["Hg"].apply(X, HX, generic=generic)
    s["Hg"].apply(Yv, HY, generic=generic)
    a = (X * HY).sum(dim=0).cpu().numpy()
    b = (HX * Yv).sum(dim=0).cpu().numpy()
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


def test_ritz_values_independent_of_basis(system):
    s = system
    B = s["B"]
    ctx = B.Context(0)
    m = 24
    X0, _ = np.linalg.qr(random_block(s["g"].n, m, 13))
    U, _ = np.linalg.qr(np.random.default_rng(14).standard_normal((m, m)))
    evs = []
    for Xh in (X0, X0 @ U):
        X = to_rows(s, Xh, torch.float64)
        W = torch.zeros_like(X)
        evs.append(B.rayleigh_ritz(s["Hg"], ctx, X, W))
    assert np.abs(evs[0] - evs[1]).max() < 1e-10 * np.abs(evs[0]).max()


def test_poisson_iteration_limit_reported(system):
    s = system
    B = s["B"]
    ctx = B.Context(0)
    rho = to_rows(s, np.exp(-((s["g"].xyz ** 2).sum(axis=1)) / 8.0), torch.float64)
    vh = torch.zeros_like(rho)
    with pytest.raises(B.ChfError) as e:
        s["Hg"].hartree(ctx, rho, vh, rtol=1e-12, max_iter=2)
    assert e.value.code == -5


def test_zero_block_is_not_positive_definite(system):
    s = system
    B = s["B"]
    ctx = B.Context(0)
    X = torch.zeros((s["Hg"].n_rows, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:
        B.orthonormalize(ctx, X)
    assert e.value.code == -4
