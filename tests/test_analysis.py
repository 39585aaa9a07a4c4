"""Post-processing of converged runs: DOS histograms and the gap fit
(Results section: 0.1 eV bins with the highest occupied state at zero,
areas normalised below it; gap(d) = E0 + A / d^k)."""
import numpy as np
import pytest

from paper_2303_00790_amd import analysis as A


def test_fit_recovers_the_published_power_law():
    # the paper's fitted constants, sampled at its cluster diameters' range
    d = np.array([1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 10.0, 16.0])
    g = 0.46 + 4.64 / d ** 1.56
    e0, a, k, r2 = A.fit_gap(d, g)
    assert abs(e0 - 0.46) < 1e-6 and abs(a - 4.64) < 1e-6 and abs(k - 1.56) < 1e-6
    assert r2 > 1 - 1e-12


def test_fit_with_noise_keeps_r2_below_one():
    rng = np.random.default_rng(0)
    d = np.linspace(1, 5, 9)
    g = 0.46 + 4.64 / d ** 1.56 + rng.normal(0, 0.01, d.size)
    *_, r2 = A.fit_gap(d, g)
    assert 0.99 < r2 < 1.0


def test_gap_in_ev():
    eig = np.array([-0.5, -0.3, -0.2, 0.1, 0.2])
    assert A.gap_ev(eig, 3) == pytest.approx(0.3 * A.HARTREE_EV)
    with pytest.raises(ValueError):
        A.gap_ev(eig, 5)


def test_dos_aligned_at_homo_and_normalised():
    rng = np.random.default_rng(1)
    eig = np.sort(rng.uniform(-0.5, 0.1, 400))
    n_occ = 300
    edges, dens = A.dos_histogram(eig, n_occ, bin_ev=0.1, lo_ev=-20, hi_ev=5, area=2.0)
    assert np.allclose(np.diff(edges), 0.1)
    # 0 eV is a bin edge and the highest occupied state is in the bin ending there
    k0 = int(np.argmin(np.abs(edges)))
    assert abs(edges[k0]) < 1e-12 and dens[k0 - 1] > 0
    assert dens[edges[1:] <= 1e-12].sum() * 0.1 == pytest.approx(2.0)
    # unnormalised counts cover every eigenvalue inside the window
    _, raw = A.dos_histogram(eig, n_occ, bin_ev=0.1, lo_ev=-20, hi_ev=5, area=n_occ * 0.1)
    assert raw.sum() == pytest.approx(eig.size, rel=1e-12)


def test_dos_rms():
    a = np.array([1.0, 2.0, 3.0])
    assert A.dos_rms(a, a) == 0.0
    assert A.dos_rms(a, a + 1) == pytest.approx(1.0)


def test_fixed_exponent_fit():
    d = np.array([1.0, 2.0, 3.0, 4.0])
    g = 0.46 + 4.64 / d ** 1.56
    e0, a, k, r2 = A.fit_gap(d, g, k=1.56)
    assert abs(e0 - 0.46) < 1e-12 and abs(a - 4.64) < 1e-12 and k == 1.56 and r2 == pytest.approx(1.0)
