"""Pins of the beam-scan oracle (paper Sec. 3.1: element positions, phase
shift, received signal, beam-scan spectrum) against closed forms."""
import numpy as np
import pytest

from oracle import beamscan as Bs


def _dirichlet(x, s):
    """|sum_{k<s} exp(j k x)| = |sin(s x / 2) / sin(x / 2)| (s where sin(x/2) = 0)."""
    x = np.asarray(x, np.float64)
    den = np.sin(0.5 * x)
    small = np.abs(den) < 1e-12
    return np.where(small, float(s), np.abs(np.sin(0.5 * s * x)) / np.where(small, 1.0, np.abs(den)))


@pytest.mark.parametrize("side,d,az0,el0", [(4, 0.5, 37, 20), (4, 0.5, 300, 71), (3, 0.35, 181, 5),
                                            (2, 0.5, 90, 0)])
def test_single_path_is_the_separable_array_factor(side, d, az0, el0):
    # One path from (theta0, phi0): the spectrum is the product of two Dirichlet
    # kernels in u = 2 pi d (cos phi cos theta - cos phi0 cos theta0) and
    # v = 2 pi d (cos phi sin theta - cos phi0 sin theta0), divided by K, since
    # r cos(theta - beta) = D ((n - 1) cos theta + (m - 1) sin theta).
    H, W = 90, 360
    th0, ph0 = np.deg2rad(az0), np.deg2rad(el0)
    paths = np.array([[0.37, th0, ph0]])
    A = Bs.spectrum(paths, 1, H, W, side, d)
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    th, ph = 2 * np.pi * xs / W, 0.5 * np.pi * ys / H
    u = 2 * np.pi * d * (np.cos(ph) * np.cos(th) - np.cos(ph0) * np.cos(th0))
    v = 2 * np.pi * d * (np.cos(ph) * np.sin(th) - np.cos(ph0) * np.sin(th0))
    ref = _dirichlet(u, side) * _dirichlet(v, side) / side ** 2
    np.testing.assert_allclose(A, ref, rtol=1e-9, atol=1e-12)
    assert A[el0, az0] == pytest.approx(1.0, abs=1e-12)


def test_power_scaling_leaves_the_spectrum_unchanged():
    rng = np.random.default_rng(1)
    paths = np.stack([rng.uniform(0.1, 1, 12), rng.uniform(0, 2 * np.pi, 12), rng.uniform(0, np.pi / 2, 12)], 1)
    a = Bs.spectrum(paths, 12, 30, 60)
    p2 = paths.copy()
    p2[:, 0] *= 7.3
    np.testing.assert_allclose(Bs.spectrum(p2, 12, 30, 60), a, rtol=1e-12, atol=1e-14)
    # and the spectrum is bounded by 1 (|sum of K unit phasors| / K)
    assert a.max() <= 1.0 + 1e-12 and a.min() >= 0.0


def test_one_element_and_no_paths():
    rng = np.random.default_rng(2)
    paths = np.stack([rng.uniform(0.1, 1, 5), rng.uniform(0, 2 * np.pi, 5), rng.uniform(0, np.pi / 2, 5)], 1)
    np.testing.assert_allclose(Bs.spectrum(paths, 5, 9, 17, side=1), 1.0, rtol=0, atol=1e-15)
    np.testing.assert_array_equal(Bs.spectrum(paths, 0, 9, 17), 0.0)


def test_reference_element_has_no_phase():
    r, beta = Bs.element_positions(4)
    assert r[0] == 0.0
    da = Bs.phase_difference(1.1, 0.3, 4)
    assert da[0] == 0.0
    # element (m, n) = (1, 2) lies along the n axis: phase -2 pi D cos(phi) cos(theta)
    assert da[1] == pytest.approx(-2 * np.pi * 0.5 * np.cos(0.3) * np.cos(1.1), rel=1e-14)
    # element (2, 1) along the m axis: -2 pi D cos(phi) sin(theta)
    assert da[4] == pytest.approx(-2 * np.pi * 0.5 * np.cos(0.3) * np.sin(1.1), rel=1e-14)
