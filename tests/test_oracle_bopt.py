"""Pins of the B_opt oracle (Algorithms 4.3 / 4.4) against definitions.

* (4.13) and (4.14) against H_l^* H_l and |I_Ms|^{-1} H_l^* D^{-1} f_l built
  entry by entry from (4.11) and the dense D, F of (2.13), (2.14);
* the column index sets against the nonzero pattern of the dense B of (2.15);
* the column-wise solution against the definition's stacked real least
  squares, on well-posed sizes (every column set much smaller than |I_M|,
  the full-column-rank case of (4.12));
* optimality: B_opt's objective (4.9) is below that of perturbed matrices of
  the same pattern and below that of the density-compensated window matrix
  W^* B of the remark opening Section 4 (a feasible point), for the weights
  of Algorithm 3.6;
* the FFT route of Algorithm 4.4 against D^* F^* B_opt^* f with dense matrices;
* planted mistakes (Dirichlet kernel with M instead of M - 1, flipped phase
  in (4.14)) each fail a pin.
"""
import math

import numpy as np
import pytest

from oracle import bopt, ndft, nfft, window, weights, metrics
from paper_2302_00414_amd import workloads as wl


def _col(x, M, sigma, m, c):
    ip, nodes = bopt.column_sets(x, M, sigma, m)
    return nodes[ip[c]:ip[c + 1]]


@pytest.mark.parametrize("d,N,M", [(1, 60, 16), (2, 200, 8), (3, 100, 4)])
def test_gram_closed_form(d, N, M):
    x = wl.uniform_nodes(N, d, 10 + d)
    K = ndft.index_set(M, d)
    js = np.arange(min(N, 25))
    H = np.exp(-2j * math.pi * (K @ x[js].T))
    G = bopt.gram(x[js], M)
    assert np.max(np.abs(G - H.conj().T @ H)) <= 1e-12 * M ** d
    # duplicated node: the diagonal value |I_M| off the diagonal as well
    G2 = bopt.gram(np.vstack([x[:1], x[:1]]), M)
    assert np.allclose(G2, M ** d)


@pytest.mark.parametrize("d,N,M,m", [(1, 50, 16, 3), (2, 120, 8, 2)])
def test_rhs_closed_form(d, N, M, m):
    sigma = 2.0
    x = wl.uniform_nodes(N, d, 20 + d)
    Ms = window.oversampled_size(M, sigma)
    K = ndft.index_set(M, d)
    L = ndft.index_set(Ms, d)
    D, F, _ = nfft.dense_matrices(x, M, sigma, m)
    ip, nodes = bopt.column_sets(x, M, sigma, m)
    for c in (0, len(ip) // 3, len(ip) - 2):
        js = nodes[ip[c]:ip[c + 1]]
        if len(js) == 0:
            continue
        H = np.exp(-2j * math.pi * (K @ x[js].T))
        ref = H.conj().T @ np.linalg.inv(D) @ F.conj().T[:, c] / Ms ** d
        v = bopt.rhs(x[js], L[c], M, sigma, m)
        assert np.max(np.abs(v - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,N,M,m", [(1, 40, 16, 2), (2, 60, 8, 2)])
def test_column_sets_are_the_pattern_of_B(d, N, M, m):
    x = np.concatenate([wl.uniform_nodes(N, d, 30 + d),
                        np.zeros((2, d)), np.full((1, d), -0.5)])   # grid-aligned nodes
    _, _, B = nfft.dense_matrices(x, M, 2.0, m)
    ip, nodes = bopt.column_sets(x, M, 2.0, m)
    for c in range(B.shape[1]):
        assert list(nodes[ip[c]:ip[c + 1]]) == list(np.nonzero(B[:, c])[0])


@pytest.mark.parametrize("d,N,M,sigma,m", [(1, 96, 64, 2.0, 2), (2, 300, 16, 1.0, 2),
                                           (2, 150, 16, 2.0, 3)])
def test_columnwise_solution_is_the_definition(d, N, M, sigma, m):
    x = wl.uniform_nodes(N, d, 40 + d)
    B = bopt.bopt(x, M, sigma, m).toarray()
    Bd = bopt.bopt_dense(x, M, sigma, m)
    # the normal equations (4.12) square the conditioning of H_l: random nodes
    # that nearly coincide make a few columns ill-conditioned, so entries agree
    # to ~kappa^2 eps and the objectives to rounding
    assert np.max(np.abs(B - Bd)) <= 1e-5 * np.max(np.abs(Bd))
    ob, od = bopt.objective(x, B, M, sigma, m), bopt.objective(x, Bd, M, sigma, m)
    assert abs(ob - od) <= 1e-8 * od + 1e-20


@pytest.mark.parametrize("d,N,M,sigma,m", [(1, 96, 32, 2.0, 2), (2, 300, 16, 1.0, 2)])
def test_objective_is_minimal(d, N, M, sigma, m):
    x = wl.uniform_nodes(N, d, 50 + d)
    B = bopt.bopt(x, M, sigma, m)
    best = bopt.objective(x, B, M, sigma, m)
    rng = np.random.default_rng(0)
    for _ in range(3):
        P = B.copy()
        P.data = P.data * (1 + 1e-3 * rng.standard_normal(P.data.shape))
        assert bopt.objective(x, P, M, sigma, m) > best
    # the density-compensated window matrix W^* B is feasible (same pattern)
    _, _, Bw = nfft.dense_matrices(x, M, sigma, m)
    w = weights.weights_lstsq(x, M)
    # W^* B: rows scaled by conj(w); the objective takes real B, so use |w|-free form:
    # compare against the real feasible matrix diag(Re w) B
    assert bopt.objective(x, np.real(w)[:, None] * Bw, M, sigma, m) >= best


@pytest.mark.parametrize("d,N,M,sigma,m", [(1, 96, 32, 2.0, 2), (2, 300, 16, 1.0, 2)])
def test_reconstruction_fft_route_and_accuracy(d, N, M, sigma, m):
    x = wl.uniform_nodes(N, d, 60 + d)
    B = bopt.bopt(x, M, sigma, m)
    fh = wl.complex_normal(M ** d, 61)
    f = ndft.forward(x, fh, M)
    h = bopt.reconstruct(x, f, B, M, sigma, m)
    D, F, _ = nfft.dense_matrices(x, M, sigma, m)
    hd = D.conj().T @ F.conj().T @ (B.toarray().T @ f)
    assert metrics.rel_err(h, hd) <= 1e-12
    # the optimized adjoint is a far better inverse than the plain adjoint NFFT
    plain = nfft.adjoint(x, f, M, sigma, m)
    assert metrics.rel_err(h, fh) < 0.1 * metrics.rel_err(plain / N * M ** d, fh)


def test_planted_mistakes_fail_the_pins(monkeypatch):
    x = wl.uniform_nodes(30, 1, 70)
    M = 16
    K = ndft.index_set(M, 1)
    H = np.exp(-2j * math.pi * (K @ x.T))
    ref = H.conj().T @ H
    # Dirichlet kernel of length M instead of M - 1
    orig_sin = np.sin

    def bad_gram(xs, M):
        s = xs[:, 0][:, None] - xs[:, 0][None, :]
        den = orig_sin(math.pi * s)
        dk = np.where(np.abs(den) < 1e-300, M, orig_sin(M * math.pi * s) / np.where(np.abs(den) < 1e-300, 1, den))
        return dk + np.exp(-1j * M * math.pi * s)

    assert np.max(np.abs(bad_gram(x, M) - ref)) > 1e-3
    assert np.max(np.abs(bopt.gram(x, M) - ref)) < 1e-10
    # flipped phase in (4.14)
    Ms = window.oversampled_size(M, 2.0)
    D, F, _ = nfft.dense_matrices(x, M, 2.0, 2)
    c = 5
    L = ndft.index_set(Ms, 1)
    vref = H.conj().T @ np.linalg.inv(D) @ F.conj().T[:, c] / Ms
    bad = np.conj(bopt.rhs(x, -L[c], M, 2.0, 2))
    assert np.max(np.abs(bad - vref)) > 1e-3 * np.max(np.abs(vref))


@pytest.mark.parametrize("d,N,M,sigma,m", [(1, 96, 32, 2.0, 2), (2, 300, 16, 1.0, 2)])
def test_inverse_adjoint_fft_route(d, N, M, sigma, m):
    """Remark 4.6: f = B_opt F D h by the FFT route equals the dense product."""
    x = wl.uniform_nodes(N, d, 80 + d)
    B = bopt.bopt(x, M, sigma, m)
    h = wl.complex_normal(M ** d, 81)
    D, F, _ = nfft.dense_matrices(x, M, sigma, m)
    f = bopt.inverse_adjoint(x, h, B, M, sigma, m)
    assert metrics.rel_err(f, B.toarray() @ (F @ (D @ h))) <= 1e-12


def test_inverse_adjoint_solves_the_adjoint_system():
    """Remark 4.6 with |I_M| <= N: A^* f ~ h for f = B_opt F D h (jittered
    grid, sigma = 2), far closer than with the window matrix B scaled by the
    best constant."""
    x = wl.jittered_nodes((24, 24), 82)
    M, sigma, m = 16, 2.0, 4
    B = bopt.bopt(x, M, sigma, m)
    h = wl.complex_normal(M * M, 83)
    f = bopt.inverse_adjoint(x, h, B, M, sigma, m)
    e_opt = metrics.rel_err(ndft.adjoint(x, f, M), h)
    fb = nfft.forward(x, h, M, sigma, m)                  # B F D h with the window matrix
    r = ndft.adjoint(x, fb, M)
    c = np.vdot(r, h) / np.vdot(r, r)
    e_plain = metrics.rel_err(c * r, h)
    assert e_opt < 0.05 and e_opt < 0.2 * e_plain


def test_single_columns_match_the_whole_matrix():
    """bopt_columns (columns solved alone, for checking large problems) gives
    the columns of bopt."""
    x = wl.uniform_nodes(300, 2, 77)
    M, sigma, m = 16, 2.0, 2
    B = bopt.bopt(x, M, sigma, m).tocsc()
    cols = [0, 5, 300, 511, 1023]
    for c, (js, vals) in bopt.bopt_columns(x, M, sigma, m, cols).items():
        s, e = B.indptr[c], B.indptr[c + 1]
        assert np.array_equal(js, B.indices[s:e])
        assert np.array_equal(vals, B.data[s:e])
