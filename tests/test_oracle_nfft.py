"""Pins for O2 (Algorithms 2.1 and 2.4 with the Kaiser-Bessel window) -- CPU only."""
import math

import numpy as np
import pytest

from oracle import ndft, nfft, window, metrics
from paper_2302_00414_amd import workloads as wl


def _nodes_with_grid_points(N, d, Ms, seed):
    """Random nodes plus a few that sit exactly on grid points (closed edge case)."""
    x = wl.uniform_nodes(N, d, seed)
    x[0] = 0.0
    x[1] = 3.0 / Ms
    x[2] = -0.5
    return x


@pytest.mark.parametrize("d,M,sigma,m,N", [
    (1, 8, 2.0, 3, 9), (1, 6, 1.5, 2, 7), (2, 4, 2.0, 2, 6), (2, 4, 1.25, 3, 5),
    (1, 2, 2.0, 2, 4),   # M_s = 4 < 2m+1: the periodised window wraps onto itself
    (3, 2, 2.0, 1, 4)])
def test_dense_factorisation(d, M, sigma, m, N):
    """A ~ B F D and A^* ~ D^* F^* B^* with D, F, B built entry by entry from
    (2.13)-(2.15): the step-by-step algorithms equal the matrix products."""
    Ms = window.oversampled_size(M, sigma)
    x = _nodes_with_grid_points(N, d, Ms, 21)
    D, F, B = nfft.dense_matrices(x, M, sigma, m)
    fh = wl.complex_normal(M ** d, 22)
    f = wl.complex_normal(N, 23)
    np.testing.assert_allclose(nfft.forward(x, fh, M, sigma, m), B @ F @ D @ fh, atol=1e-12)
    np.testing.assert_allclose(nfft.adjoint(x, f, M, sigma, m),
                               D.conj().T @ F.conj().T @ B.T @ f, rtol=1e-12, atol=1e-12)


def test_window_error_decay():
    """P11 / S18: against the exact sums the KB NFFT error falls geometrically
    in m (sigma = 2). Measured values at d = 2, M = 32, N = 4096 random nodes
    are 2.7e-4, 3.0e-6, 3.6e-8, 4.2e-10, 5.0e-12, 6.1e-14, 4.2e-15 (adjoint,
    m = 2..8); m >= 6 is needed for 1e-10 against the exact sums."""
    x = wl.uniform_nodes(4096, 2, 1)
    fh = wl.complex_normal(32 * 32, 2)
    f = ndft.forward(x, fh, 32)
    h = ndft.adjoint(x, f, 32)
    errs = [metrics.rel_err(nfft.adjoint(x, f, 32, 2.0, m), h) for m in range(2, 9)]
    errs_f = [metrics.rel_err(nfft.forward(x, fh, 32, 2.0, m), f) for m in range(2, 9)]
    for e in (errs, errs_f):
        for a, b in zip(e[:-2], e[1:-1]):
            assert b < a / 30.0          # each extra m gains a factor > 30
        assert e[0] < 1e-3 and e[4] < 1e-10 and e[6] < 1e-13


@pytest.mark.parametrize("d", [1, 2, 3])
def test_shift_by_grid_cells(d):
    """P8: shifting every node by v/M_s (integer v) multiplies the adjoint
    output by exp(-2 pi i k.v/M_s) -- exact for the NFFT, not only for A^*."""
    M, sigma, m = 8, 2.0, 3
    Ms = window.oversampled_size(M, sigma)
    x = wl.uniform_nodes(60, d, 30 + d)
    f = wl.complex_normal(60, 31)
    v = np.array([3, -5, 7][:d], dtype=np.float64)
    base = nfft.adjoint(x, f, M, sigma, m)
    shifted = nfft.adjoint(x + v / Ms, f, M, sigma, m)
    K = ndft.index_set(M, d)
    np.testing.assert_allclose(shifted, base * np.exp(-2j * math.pi * K @ v / Ms),
                               rtol=1e-11, atol=1e-11 * np.abs(base).max())


@pytest.mark.parametrize("d,M", [(1, 16), (2, 8), (3, 4)])
def test_adjointness(d, M):
    """P6 at oracle level: <B F D fhat, g> = <fhat, D^* F^* B^* g>."""
    x = wl.uniform_nodes(100, d, 40)
    fh = wl.complex_normal(M ** d, 41)
    g = wl.complex_normal(100, 42)
    lhs = np.vdot(g, nfft.forward(x, fh, M, 2.0, 4))
    rhs = np.vdot(nfft.adjoint(x, g, M, 2.0, 4), fh)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_multiple_rhs_equal_separate():
    x = wl.uniform_nodes(200, 2, 50)
    F = wl.complex_normal((3, 200), 51)
    both = nfft.adjoint(x, F, 8, 2.0, 4)
    for r in range(3):
        np.testing.assert_allclose(both[r], nfft.adjoint(x, F[r], 8, 2.0, 4), atol=1e-13)


def test_equispaced_reconstruction_through_nfft():
    """P1 through the NFFT: equispaced nodes with w = 1/N reconstruct fhat to
    the window error (nodes sit on grid points, so the closed edge counts)."""
    x = wl.equispaced_nodes(32, 2)
    fh = wl.complex_normal(16 * 16, 52)
    f = ndft.forward(x, fh, 16)
    rec = nfft.adjoint(x, f / x.shape[0], 16, 2.0, 6)
    assert metrics.rel_err(rec, fh) < 1e-10


def test_planted_fft_direction_error_is_caught(monkeypatch):
    """Using the inverse FFT in step 2 of Alg. 2.4 breaks agreement with O1."""
    monkeypatch.setattr(np.fft, "fftn", lambda a, axes=None: np.fft.ifftn(a, axes=axes) * np.prod([a.shape[i] for i in axes]))
    x = wl.uniform_nodes(300, 2, 60)
    f = wl.complex_normal(300, 61)
    assert metrics.rel_err(nfft.adjoint(x, f, 8, 2.0, 6), ndft.adjoint(x, f, 8)) > 1e-2


def test_planted_dropped_edge_is_caught(monkeypatch):
    """Evaluating only 2m cells per dimension (dropping the closed edge)
    breaks the dense factorisation on grid-aligned nodes."""
    orig = nfft._footprint

    def short(x, Ms, m, sigma):
        ell, val = orig(x, Ms, m, sigma)
        val = val.copy()
        val[:, :, 0] = 0.0
        return ell, val
    monkeypatch.setattr(nfft, "_footprint", short)
    M, sigma, m = 4, 2.0, 2
    x = _nodes_with_grid_points(5, 1, 8, 70)
    D, F, B = nfft.dense_matrices(x, M, sigma, m)
    f = wl.complex_normal(5, 71)
    assert not np.allclose(nfft.adjoint(x, f, M, sigma, m), D.conj().T @ F.conj().T @ B.T @ f,
                           rtol=1e-12, atol=1e-12)
