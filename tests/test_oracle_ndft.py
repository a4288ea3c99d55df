"""Pins for O1 (the direct sums (2.5)/(2.6)) -- CPU only."""
import math
import os

import numpy as np
import pytest

from oracle import ndft, metrics
from paper_2302_00414_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ndft_tiny.txt")


def _golden_cases():
    cases = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        name, kind, d, M, nodes, inp, exp = [p.strip() for p in line.split("|")]
        x = np.array([[float(c) for c in pt.split(",")] for pt in nodes.split(";")])
        cases.append((name, kind, int(d), int(M), x,
                      np.array([complex(v) for v in inp.split(";")]),
                      np.array([complex(v) for v in exp.split(";")])))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c[0])
def test_hand_derived_values(case):
    """Worked values of (2.5)/(2.6): pin sign, index order and C order."""
    _, kind, d, M, x, inp, exp = case
    fn = ndft.adjoint if kind == "adjoint" else ndft.forward
    got = fn(x, inp, M)
    np.testing.assert_allclose(got, exp, atol=1e-14)
    loops = ndft.adjoint_loops if kind == "adjoint" else ndft.forward_loops
    np.testing.assert_allclose(loops(x, inp, M), exp, atol=1e-14)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_single_node_closed_form(d):
    """P7: one node, f = 1 => h_k = exp(-2 pi i k.x)."""
    x = wl.uniform_nodes(1, d, 11 + d)
    M = 6
    h = ndft.adjoint(x, np.ones(1), M)
    K = ndft.index_set(M, d)
    np.testing.assert_allclose(h, np.exp(-2j * math.pi * K @ x[0]), atol=1e-14)


@pytest.mark.parametrize("d,M,N", [(1, 8, 7), (2, 4, 9), (3, 2, 5)])
def test_vectorised_equals_loops(d, M, N):
    x = wl.uniform_nodes(N, d, 3)
    f = wl.complex_normal(N, 4)
    fh = wl.complex_normal(M ** d, 5)
    np.testing.assert_allclose(ndft.adjoint(x, f, M), ndft.adjoint_loops(x, f, M), atol=1e-12)
    np.testing.assert_allclose(ndft.forward(x, fh, M), ndft.forward_loops(x, fh, M), atol=1e-12)


@pytest.mark.parametrize("d,M,N", [(1, 16, 50), (2, 8, 300), (3, 4, 200)])
def test_adjointness(d, M, N):
    """<A fhat, g> = <fhat, A^* g> for the forward and adjoint sums."""
    x = wl.uniform_nodes(N, d, 6)
    fh = wl.complex_normal(M ** d, 7)
    g = wl.complex_normal(N, 8)
    lhs = np.vdot(g, ndft.forward(x, fh, M))
    rhs = np.vdot(ndft.adjoint(x, g, M), fh)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("d,n,M", [(1, 16, 16), (1, 20, 8), (2, 8, 8), (2, 10, 6), (3, 6, 4)])
def test_equispaced_exact_inversion(d, n, M):
    """P1, (3.1): equispaced x = j/n with n >= M and w = 1/N gives
    A^* W A = I, i.e. exact reconstruction of any trigonometric polynomial."""
    x = wl.equispaced_nodes(n, d)
    N = x.shape[0]
    fh = wl.complex_normal(M ** d, 9)
    f = ndft.forward(x, fh, M)
    rec = ndft.adjoint(x, f / N, M)
    assert metrics.rel_err(rec, fh) < 1e-13


def test_matrix_form():
    """A from (2.7) reproduces both sums."""
    x = wl.uniform_nodes(13, 2, 10)
    A = ndft.fourier_matrix(x, 4)
    f = wl.complex_normal(13, 1)
    fh = wl.complex_normal(16, 2)
    np.testing.assert_allclose(A.conj().T @ f, ndft.adjoint(x, f, 4), atol=1e-12)
    np.testing.assert_allclose(A @ fh, ndft.forward(x, fh, 4), atol=1e-12)


def test_periodic_in_nodes():
    """A is 1-periodic in each coordinate: integer shifts change nothing."""
    x = wl.uniform_nodes(40, 2, 12)
    f = wl.complex_normal(40, 13)
    shift = np.array([3.0, -2.0])
    np.testing.assert_allclose(ndft.adjoint(x + shift, f, 8), ndft.adjoint(x, f, 8), atol=1e-11)


def test_sampled_outputs_match_full():
    x = wl.uniform_nodes(500, 2, 14)
    f = wl.complex_normal((2, 500), 15)
    full = ndft.adjoint(x, f, 8)
    K = ndft.index_set(8, 2)
    sel = np.array([0, 5, 17, 63])
    np.testing.assert_allclose(ndft.adjoint_at(x, f, K[sel]), full[:, sel], atol=1e-11)
    rows = [0, 7, 499]
    fh = wl.complex_normal(64, 16)
    np.testing.assert_allclose(ndft.forward_at(x, fh, 8, rows), ndft.forward(x, fh, 8)[rows], atol=1e-11)


def test_planted_sign_error_is_caught(monkeypatch):
    """A flipped exponent sign in the phase tables must break the hand-derived pins."""
    orig = ndft._phase_tables
    monkeypatch.setattr(ndft, "_phase_tables", lambda x, M: [np.conj(t) for t in orig(x, M)])
    name, kind, d, M, x, inp, exp = _golden_cases()[0]
    assert not np.allclose(ndft.adjoint(x, inp, M), exp, atol=1e-6)


def test_planted_index_order_error_is_caught(monkeypatch):
    """Enumerating I_M from +M/2 down (a reversed index set) breaks the pins."""
    monkeypatch.setattr(ndft, "freqs", lambda M: np.arange(M // 2 - 1, -M // 2 - 1, -1))
    name, kind, d, M, x, inp, exp = _golden_cases()[0]
    assert not np.allclose(ndft.adjoint(x, inp, M), exp, atol=1e-6)
