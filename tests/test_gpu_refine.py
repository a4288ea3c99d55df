"""Weighted iterative refinement on the GPU (nfft_refine) against the oracle
O5 with the reference NFFT (O2) as A and A^*, and its convergence.

* Parity: fhat_k and the relative residuals ||f - A fhat_k|| / ||f|| for
  k = 0..iters, d = 1, 2, 3, float64 and float32, one and three right-hand
  sides, on jittered grids with weights 1/N, at sizes spanning several tiles;
  and at the full polar 512 x 512, M = 256 size in the benchmark's
  configuration (float32, autotuned, 4 steps).
* iters = 0 is the plain weighted adjoint.
* Convergence with the weights of Algorithm 3.6 where the direct method is
  not exact: for samples of a trigonometric polynomial the error falls with
  every step, the residuals too.
* Argument checks (iters outside 0..1000, nrhs, missing weights).
"""
import numpy as np
import pytest
import torch

from oracle import nfft as onfft, metrics, refine as orf
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL = {"f64": 1e-12, "f32": 1e-5}
RES_TOL = {"f64": 1e-10, "f32": 1e-5}
ORDER = {"f64": 1e-13, "f32": 1e-6}
CASES = {1: ((300,), 128, 8), 2: ((48, 48), 32, 6), 3: ((20, 20, 20), 16, 4)}


def _plan(x, M, m, prec, max_rhs):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] refine N={x.shape[0]} d={x.shape[1]} M={M} m={m} {prec} rhs={max_rhs}", flush=True)
    return Plan(x, M, 2.0, m, precision=prec, max_rhs=max_rhs, device="cuda:0")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("nrhs,iters", [(1, 0), (1, 3), (3, 1), (3, 4)])
def test_refine_matches_oracle(d, nrhs, iters, prec):
    n, M, m = CASES[d]
    x = wl.jittered_nodes(n, 20 + d, jitter=0.3)
    N = x.shape[0]
    w = np.full(N, 1.0 / N, dtype=np.complex128)
    f = wl.complex_normal((nrhs, N), 21 + d)
    p = _plan(x, M, m, prec, nrhs)
    p.set_weights(w)
    got, res = p.refine(torch.from_numpy(f), iters, residuals=True)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want, wres = orf.refine(x, f, w, M, iters, op="nfft", sigma=2.0, m=m)
    assert metrics.rel_err(got, want) <= TOL[prec]
    assert res.shape == (iters + 1,)
    assert np.allclose(res, wres, rtol=RES_TOL[prec], atol=0)
    # without residuals: the same iterate (float64 spreading adds with LDS
    # atomics, so two runs agree up to rounding order)
    again = p.refine(torch.from_numpy(f), iters).cpu().numpy()
    assert metrics.rel_err(again, got) <= ORDER[prec]
    if iters == 0:
        plain = p.adjoint(torch.from_numpy(f)).cpu().numpy()
        assert metrics.rel_err(plain, got) <= ORDER[prec]
    p.close()


def test_refine_converges_with_algorithm_3_6_weights():
    """Uniform nodes with |I_M| < N < |I_2M| (the least-squares branch (3.16),
    where the direct reconstruction is not exact): with the weights of
    Algorithm 3.6 the error in the coefficients of a trigonometric polynomial
    falls with every step, and so does the residual."""
    from paper_2302_00414_amd.nfft import compute_weights
    M, m, N = 32, 6, 3000
    x = wl.uniform_nodes(N, 2, 33)
    w, info = compute_weights(x, M, 2.0, 8, 1e-13, 2000, device="cuda:0")
    assert info["branch"] == "3.16"
    fh = wl.complex_normal(M * M, 30)
    f = onfft.forward(x, fh, M, 2.0, m)
    p = _plan(x, M, m, "f64", 1)
    p.set_weights(w.cpu().numpy())
    errs = [metrics.rel_err(p.refine(torch.from_numpy(f), k).cpu().numpy(), fh)
            for k in (0, 1, 2, 4, 8, 32)]
    _, res = p.refine(torch.from_numpy(f), 8, residuals=True)
    print("[errors]", errs, "[residuals]", res.tolist(), flush=True)
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 0.5 * errs[0]
    assert all(b < a for a, b in zip(res, res[1:]))
    p.close()


def test_refine_argument_checks():
    from paper_2302_00414_amd.nfft import NfftError
    x = wl.uniform_nodes(200, 2, 31)
    p = _plan(x, 16, 4, "f64", 2)
    f = torch.zeros((2, 200), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(NfftError) as e:
        p.refine(f, 2)                     # no weights yet
    assert e.value.status == 4
    p.set_weights(np.full(200, 1 / 200, dtype=np.complex128))
    for iters in (-1, 1001):
        with pytest.raises(NfftError) as e:
            p.refine(f, iters)
        assert e.value.status == 1
    out = p.refine(f, 2)
    assert out.shape == (2, 256) and float(out.abs().max()) == 0.0
    p.close()


def test_refine_polar_512x512_M256_in_the_benchmark_configuration():
    """The refinement as the benchmark times it: polar grid R = T = 512
    (N = 262144, eq. (5.2)), M = 256, m = 6, area weights, float32, autotuned
    launch configuration, 4 steps, against O5 on the reference NFFT (whole
    iterate and every residual)."""
    from paper_2302_00414_amd.nfft import Plan
    x = wl.polar_nodes(512, 512)
    N = x.shape[0]
    w = wl.polar_area_weights(512, 512).astype(np.complex128)
    f = wl.complex_normal(N, 31)
    print(f"[case] refine polar 512x512 N={N} M=256 m=6 f32 tuning=auto iters=4", flush=True)
    p = Plan(x, 256, 2.0, 6, precision="f32", device="cuda:0", tuning="auto")
    p.set_weights(w)
    got, res = p.refine(torch.from_numpy(f), 4, residuals=True)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    p.close()
    want, wres = orf.refine(x, f, w, 256, 4, op="nfft", sigma=2.0, m=6)
    assert metrics.rel_err(got, want) <= TOL["f32"]
    assert np.allclose(res, wres, rtol=RES_TOL["f32"], atol=0)
