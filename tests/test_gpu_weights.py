"""Algorithm 3.6 on the GPU (float64 conjugate gradients on (3.15)/(3.16)
with the library's NFFT at 2M) against what the paper and the oracle fix.

* P2: on an equispaced grid of n^d nodes with n > M the weights are 1/N,
  in both branches.
* Dense agreement: the minimum-norm least-squares solution of
  A_2M^T w = e_0 by the oracle's dense solve.
* P3 (Corollary 3.4): with |I_2M| < N the weighted adjoint reconstructs
  trigonometric polynomials of degree M exactly.
* P4 (bound (3.37)): e_2 <= |I_M| epsilon.
"""
import numpy as np
import pytest
import torch

from oracle import ndft, weights as ow, metrics
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _weights(x, M, m=None, tol=1e-13, maxit=2000):
    """m = 8 (window error ~1e-15) where the float64 3-D tile allows, else 6."""
    from paper_2302_00414_amd.nfft import compute_weights
    if m is None:
        m = 8 if x.shape[1] < 3 else 6
    print(f"[case] weights N={x.shape[0]} d={x.shape[1]} M={M} m={m}", flush=True)
    w, info = compute_weights(x, M, 2.0, m, tol, maxit, device="cuda:0")
    torch.cuda.synchronize()
    print("[info]", info, flush=True)
    return w.cpu().numpy(), info


@pytest.mark.parametrize("d,n,M,branch", [(2, 48, 16, "3.15"), (2, 24, 16, "3.16"),
                                          (1, 300, 64, "3.15"), (3, 12, 8, "3.16")])
def test_equispaced_weights_are_one_over_N(d, n, M, branch):
    x = wl.equispaced_nodes(n, d)
    N = x.shape[0]
    w, info = _weights(x, M)
    assert info["branch"] == branch
    tol = 1e-12 if d < 3 else 1e-9   # NFFT window error at m = 8 / m = 6
    assert np.max(np.abs(w - 1.0 / N)) <= tol / N
    assert info["epsilon"] <= tol


@pytest.mark.parametrize("d,N,M,branch", [(2, 4096, 16, "3.15"), (2, 700, 16, "3.16"),
                                          (1, 500, 64, "3.15"), (1, 100, 64, "3.16"),
                                          (3, 3000, 4, "3.15")])
def test_matches_dense_min_norm_lstsq(d, N, M, branch):
    x = wl.uniform_nodes(N, d, 400 + d)
    w, info = _weights(x, M)
    assert info["branch"] == branch
    ref = ow.weights_lstsq(x, M)
    eps_ref = ow.residual(x, ref, M)
    if branch == "3.15":
        # consistent system: the minimum-norm solution is unique
        assert metrics.rel_err(w, ref) <= (1e-9 if d < 3 else 1e-7)
        assert info["epsilon"] <= (1e-10 if d < 3 else 1e-8)
    else:
        # least squares: the residual is that of the dense solution
        assert info["epsilon"] <= 1.01 * eps_ref + 1e-12
    # epsilon as the oracle evaluates it from the exact sums
    assert abs(ow.residual(x, w, M) - info["epsilon"]) <= 1e-9 + 1e-6 * info["epsilon"]


def test_exact_reconstruction_and_error_bound():
    from paper_2302_00414_amd.nfft import Plan
    M = 16
    for N, exact in ((4096, True), (700, False)):
        x = wl.uniform_nodes(N, 2, 410)
        w, info = _weights(x, M)
        fh = wl.complex_normal(M * M, 411)
        f = ndft.forward(x, fh, M)
        p = Plan(x, M, 2.0, 8, precision="f64", device="cuda:0")
        p.set_weights(w)
        rec = p.adjoint(torch.from_numpy(f)).cpu().numpy()
        p.close()
        e2 = metrics.rel_err(rec, fh)
        print(f"[recon] N={N} e2={e2:.3e} eps={info['epsilon']:.3e}", flush=True)
        assert e2 <= (M * M) * info["epsilon"] + 1e-12        # (3.37)
        if exact:
            assert e2 <= 1e-10                                # Corollary 3.4


@pytest.mark.parametrize("d,N,M", [(1, 300, 32), (2, 800, 16)])
def test_relaxed_and_pcf_weights_match_oracle(d, N, M):
    """The literature schemes of Section 3.4 on the GPU against the oracle:
    (3.63) A A^* w = 1 by CG, and the PCF weights (3.62)."""
    from paper_2302_00414_amd.nfft import compute_weights
    x = wl.uniform_nodes(N, d, 420 + d)
    print(f"[case] relaxed/pcf N={N} d={d} M={M}", flush=True)
    w_r, info_r = compute_weights(x, M, 2.0, 8, 1e-13, 3000, device="cuda:0", scheme="relaxed")
    w_p, info_p = compute_weights(x, M, device="cuda:0", scheme="pcf")
    w_r, w_p = w_r.cpu().numpy(), w_p.cpu().numpy()
    print("[info]", info_r, info_p, flush=True)
    assert info_r["branch"] == "3.63" and info_p["branch"] == "3.62"
    H = ow.gram_nodes(x, M)
    assert np.max(np.abs(H @ w_r - 1)) <= 1e-8
    assert info_r["epsilon"] <= 1e-8
    assert metrics.rel_err(w_p, ow.weights_pcf(x, M)) <= 1e-12
