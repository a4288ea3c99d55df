"""O5 (weighted iterative refinement) against what the paper and the algebra
fix, with exact sums (O1) for A and A^*:

* with A^* W A = I + E and q = |I_M| eps < 1 (eps the residual (3.36) of the
  weights), samples of a trigonometric polynomial are reconstructed with
  error ||fhat - fhat_k||_2 <= q^(k+1) ||fhat||_2 (k = 0 is the bound (3.37));
* the iterates tend to the weighted least-squares solution
  (A^* W A)^{-1} A^* W f (a dense solve) for any data;
* fhat_k equals the partial Neumann sum sum_{n<=k} (I - A^* W A)^n A^* W f of
  the proof of Theorem 3.15 (dense matrix powers);
* on an equispaced grid with w = 1/N (A^* W A = I) nothing is left to refine;
* the reference NFFT (O2) in place of the exact sums changes nothing beyond
  its own error.
"""
import numpy as np
import pytest

from oracle import ndft, weights, metrics, refine as orf
from paper_2302_00414_amd import workloads as wl


def _perturbed_weights(x, M, pert, seed):
    w = weights.weights_lstsq(x, M) + pert * wl.complex_normal(x.shape[0], seed)
    q = weights.residual(x, w, M) * M ** x.shape[1]
    return w, q


@pytest.mark.parametrize("d,N,M,pert", [(1, 256, 32, 2e-4), (2, 1024, 8, 6e-5), (2, 600, 6, 2e-4)])
def test_error_contracts_by_the_bound(d, N, M, pert):
    x = wl.uniform_nodes(N, d, 500 + N)
    w, q = _perturbed_weights(x, M, pert, 7)
    assert 0.1 < q < 0.9
    fh = wl.complex_normal(M ** d, 501)
    f = ndft.forward(x, fh, M)
    errs = [metrics.rel_err(orf.refine(x, f, w, M, k)[0], fh) for k in range(5)]
    for k, e in enumerate(errs):
        assert e <= q ** (k + 1) * (1 + 1e-9) + 1e-14, (k, e, q)
    assert errs[-1] < 0.1 * errs[0]


@pytest.mark.parametrize("d,N,M,pert", [(1, 256, 32, 2e-4), (2, 1024, 8, 6e-5)])
def test_limit_is_weighted_least_squares(d, N, M, pert):
    x = wl.uniform_nodes(N, d, 600 + N)
    w, q = _perturbed_weights(x, M, pert, 8)
    f = wl.complex_normal(N, 601)                 # not samples of a polynomial
    A = ndft.fourier_matrix(x, M)
    AhW = A.conj().T * w[None, :]
    ls = np.linalg.solve(AhW @ A, AhW @ f)
    K = int(np.ceil(np.log(1e-15) / np.log(q)))
    got, res = orf.refine(x, f, w, M, K)
    assert metrics.rel_err(got, ls) <= 1e-10
    # the residual of the limit is that of the least-squares solution
    assert res[-1] == pytest.approx(np.linalg.norm(f - A @ ls) / np.linalg.norm(f), rel=1e-8)


def test_iterates_are_partial_neumann_sums():
    x = wl.uniform_nodes(300, 2, 700)
    M = 6
    w, _ = _perturbed_weights(x, M, 2e-4, 9)
    f = wl.complex_normal((2, 300), 701)
    A = ndft.fourier_matrix(x, M)
    T = A.conj().T @ (w[:, None] * A)
    S = np.eye(M * M) - T
    b = (A.conj().T @ (w[None, :] * f).T).T        # A^* W f, one row per rhs
    for k in range(4):
        want = sum(np.linalg.matrix_power(S, n) @ b.T for n in range(k + 1)).T
        assert metrics.rel_err(orf.refine(x, f, w, M, k)[0], want) <= 1e-12


def test_equispaced_grid_needs_no_refinement():
    n, M = 12, 8
    x = wl.equispaced_nodes(n, 2)
    N = x.shape[0]
    w = np.full(N, 1.0 / N, dtype=np.complex128)
    f = wl.complex_normal(N, 702)
    h0, r0 = orf.refine(x, f, w, M, 0)
    h3, r3 = orf.refine(x, f, w, M, 3)
    assert metrics.rel_err(h3, h0) <= 1e-13
    assert np.allclose(r3, r0[0], rtol=1e-12)


def test_nfft_operators_match_exact_sums():
    x = wl.uniform_nodes(1024, 2, 703)
    M = 8
    w, _ = _perturbed_weights(x, M, 6e-5, 10)
    f = wl.complex_normal((2, 1024), 704)
    a, ra = orf.refine(x, f, w, M, 3, op="ndft")
    b, rb = orf.refine(x, f, w, M, 3, op="nfft", sigma=2.0, m=8)
    assert metrics.rel_err(b, a) <= 1e-11
    assert np.allclose(rb, ra, rtol=1e-9)
