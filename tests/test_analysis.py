"""Post-processing of converged runs: DOS histograms and the gap fit
(Results section: 0.1 eV bins with the highest occupied state at zero,
areas normalised below it; gap(d) = E0 + A / d^k)."""
import numpy as np
import pytest

from paper_2303_00790_amd import analysis as A
from golden import text_figures

FIG = text_figures()
E0, AMP, K = FIG["gap_offset_ev"], FIG["gap_amplitude_ev"], FIG["gap_exponent"]


def test_fit_recovers_the_published_power_law():
    # the paper's fitted constants, sampled at its cluster diameters' range
    d = np.array([1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 10.0, 16.0])
    g = E0 + AMP / d ** K
    e0, a, k, r2 = A.fit_gap(d, g)
    assert abs(e0 - E0) < 1e-6 and abs(a - AMP) < 1e-6 and abs(k - K) < 1e-6
    assert r2 > 1 - 1e-12


def test_fit_with_noise_keeps_r2_below_one():
    rng = np.random.default_rng(0)
    d = np.linspace(1, 5, 9)
    g = E0 + AMP / d ** K + rng.normal(0, 0.01, d.size)
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
    w = FIG["dos_bin_ev"]
    edges, dens = A.dos_histogram(eig, n_occ, bin_ev=w, lo_ev=-20, hi_ev=5, area=2.0)
    assert np.allclose(np.diff(edges), w)
    # 0 eV is a bin edge and the highest occupied state is in the bin ending there
    k0 = int(np.argmin(np.abs(edges)))
    assert abs(edges[k0]) < 1e-12 and dens[k0 - 1] > 0
    assert dens[edges[1:] <= 1e-12].sum() * w == pytest.approx(2.0)
    # unnormalised counts cover every eigenvalue inside the window
    _, raw = A.dos_histogram(eig, n_occ, bin_ev=w, lo_ev=-20, hi_ev=5, area=n_occ * w)
    assert raw.sum() == pytest.approx(eig.size, rel=1e-12)


def test_default_bin_is_the_papers():
    assert A.dos_histogram.__defaults__[0] == FIG["dos_bin_ev"]


def test_dos_rms():
    a = np.array([1.0, 2.0, 3.0])
    assert A.dos_rms(a, a) == 0.0
    assert A.dos_rms(a, a + 1) == pytest.approx(1.0)


def test_fixed_exponent_fit():
    d = np.array([1.0, 2.0, 3.0, 4.0])
    g = E0 + AMP / d ** K
    e0, a, k, r2 = A.fit_gap(d, g, k=K)
    assert abs(e0 - E0) < 1e-12 and abs(a - AMP) < 1e-12 and k == K and r2 == pytest.approx(1.0)
