"""Pins for the Kaiser-Bessel window pair of the oracle -- CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import window


@pytest.mark.parametrize("M,sigma,Ms", [(32, 2.0, 64), (10, 1.5, 16), (10, 1.25, 14),
                                        (8, 1.0, 8), (7 * 2, 1.1, 16), (256, 2.0, 512)])
def test_oversampled_size(M, sigma, Ms):
    """M_sigma = 2 ceil(ceil(sigma M)/2), worked by hand."""
    assert window.oversampled_size(M, sigma) == Ms


@pytest.mark.parametrize("m", [2, 4, 6, 8])
def test_edge_value_and_support(m):
    """w_m keeps the closed cube: value b/pi at |t| = m, zero beyond."""
    b = window.shape_b(2.0)
    np.testing.assert_allclose(window.phi(np.array([-m, m]), m, 2.0), b / math.pi, rtol=1e-15)
    assert np.all(window.phi(np.array([m + 1e-12, -m - 1e-9, 7.0 * m]), m, 2.0) == 0.0)
    t = np.linspace(-m, m, 41)
    np.testing.assert_allclose(window.phi(t, m, 2.0), window.phi(-t, m, 2.0), rtol=1e-15)


@pytest.mark.parametrize("m,sigma", [(4, 2.0), (6, 2.0), (3, 1.5), (8, 1.25)])
def test_fourier_pair_by_quadrature(m, sigma):
    """P10: w(x) = int hat w(k) exp(2 pi i k x) dk. hat w is supported on
    |k| <= M_s b / (2 pi), so the inverse transform is a finite integral that
    adaptive (cosine-weighted) quadrature evaluates to ~1e-15 of w(0)."""
    Ms = 64
    b = window.shape_b(sigma)
    K = Ms * b / (2 * math.pi)
    p0 = float(window.phi(0.0, m, sigma))
    f = lambda k: 2 * window.phi_hat(np.array([k]), m, sigma, Ms)[0]
    for t in [0.0, 0.3, 1.7, m - 0.5, m - 1e-3]:
        x = t / Ms
        if x == 0.0:
            val, _ = integrate.quad(f, 0.0, K, limit=400, epsabs=0, epsrel=1e-13)
        else:
            val, _ = integrate.quad(f, 0.0, K, weight="cos", wvar=2 * math.pi * x,
                                    limit=400, epsabs=1e-14 * p0)
        assert abs(val - float(window.phi(t, m, sigma))) <= 1e-13 * p0


def test_untruncated_window_continuity():
    """The untruncated window joins its sinh and sin branches at |t| = m."""
    m, s = 4, 2.0
    t = np.array([m - 1e-7, m, m + 1e-7])
    v = window.phi_full(t, m, s)
    np.testing.assert_allclose(v, v[1], rtol=1e-5)


def test_planted_normalisation_error_is_caught(monkeypatch):
    """Dropping the 1/M_s of hat w breaks the quadrature pin."""
    orig = window.phi_hat
    monkeypatch.setattr(window, "phi_hat", lambda k, m, s, Ms: orig(k, m, s, Ms) * Ms)
    m, sigma, Ms = 4, 2.0, 64
    K = Ms * window.shape_b(sigma) / (2 * math.pi)
    val, _ = integrate.quad(lambda k: 2 * window.phi_hat(np.array([k]), m, sigma, Ms)[0], 0.0, K)
    assert abs(val - float(window.phi(0.0, m, sigma))) > 1e-3 * abs(val)


@pytest.mark.parametrize("m,sigma", [(4, 2.0), (6, 2.0), (8, 2.0), (3, 1.25)])
def test_window_values_to_float64_rounding(m, sigma):
    """The window's values against a 40-digit evaluation of its definition
    sinh(b sqrt(m^2 - t^2)) / (pi sqrt(m^2 - t^2)) (mpmath): within 2 units
    in the last place at every offset, so the oracle's window adds no error
    beyond float64 rounding to the sums it enters."""
    import mpmath as mp
    mp.mp.dps = 40
    b = mp.pi * (2 - mp.mpf(1) / mp.mpf(sigma))
    rng = np.random.default_rng(m)
    t = np.concatenate([rng.uniform(-m, m, 400), np.linspace(-m, m, 101)])
    got = window.phi(t, m, sigma)
    for tv, g in zip(t, got):
        z = mp.sqrt(m * m - mp.mpf(float(tv)) ** 2)
        ex = mp.sinh(b * z) / (mp.pi * z) if z > 0 else b / mp.pi
        assert abs(g - float(ex)) <= 2 * np.spacing(float(ex)), (tv, g, float(ex))
