"""Example 5.5 on the GPU at the paper's size: the band-limited triangular
pulse with b = 24, M = 64, on the jittered 144 x 144 grid (|I_2M| <= N).

Reconstructions of the samples fhat(k), k in I_M, compared by their largest
pointwise error, as the example does:
* Algorithm 3.7 with the weights of Algorithm 3.6 (the second-kind normal
  equations (3.15), as |I_2M| <= N) and Algorithm 4.4 with the optimized
  sparse matrix both match the error of a reconstruction from an equispaced
  144 x 144 grid, the best possible here (the truncation error of the
  integral dominates);
* the PCF weights (3.62), the relaxed weights (3.63) and plain 1/N weights
  do clearly worse.
The equispaced reconstruction itself is checked against the oracle's NFFT.
Algorithm 4.4 runs at sigma = 2, m = 4: at sigma = 1 a grid column of this
node density holds more nodes than the library's column solve takes.
"""
import numpy as np
import pytest
import torch

from oracle import nfft as onfft, metrics
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

M, B, NG = 64, 24, 144


def _adjoint(x, f, w, m=6):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] adjoint N={x.shape[0]} M={M} m={m}", flush=True)
    p = Plan(x, M, 2.0, m, precision="f64", device="cuda:0")
    p.set_weights(w)
    h = p.adjoint(torch.from_numpy(f).to("cuda:0"))
    torch.cuda.synchronize()
    p.close()
    return h.cpu().numpy()


@pytest.fixture(scope="module")
def errors():
    from paper_2302_00414_amd.nfft import Plan, compute_weights
    fh = wl.triangle_pulse_coefficients(M, 2, B)

    def err(h):
        return float(np.max(np.abs(h - fh)))

    out = {}
    xe = wl.equispaced_nodes(NG, 2)
    fe = wl.triangle_pulse_samples(xe, B)
    we = np.full(xe.shape[0], 1.0 / xe.shape[0], dtype=np.complex128)
    he = _adjoint(xe, fe, we)
    out["equispaced_vs_oracle"] = metrics.rel_err(he, onfft.adjoint(xe, we * fe, M, 2.0, 6))
    out["equispaced"] = err(he)

    x = wl.jittered_nodes((NG, NG), 5, jitter=1.0)
    N = x.shape[0]
    assert (2 * M) ** 2 <= N
    f = wl.triangle_pulse_samples(x, B)
    for scheme in ("alg3.6", "pcf", "relaxed"):
        print(f"[case] weights {scheme}", flush=True)
        w, info = compute_weights(x, M, 2.0, 8, 1e-13, 2000, device="cuda:0", scheme=scheme)
        out[scheme] = err(_adjoint(x, f, w.cpu().numpy()))
        out[scheme + "_branch"] = info["branch"]
    out["one_over_n"] = err(_adjoint(x, f, np.full(N, 1.0 / N, dtype=np.complex128)))

    print("[case] optimized sparse matrix sigma=2 m=4", flush=True)
    p = Plan(x, M, 2.0, 4, precision="f64", device="cuda:0")
    info = p.build_bopt(x)
    assert info["singular_columns"] == 0
    out["bopt"] = err(p.bopt_adjoint(torch.from_numpy(f).to("cuda:0")).cpu().numpy())
    p.close()
    print("[errors]", out, flush=True)
    return out


def test_equispaced_reference(errors):
    assert errors["equispaced_vs_oracle"] <= 1e-12
    assert errors["equispaced"] > 1e-2  # the truncation error of the integral


def test_weights_and_optimized_matrix_match_the_grid(errors):
    assert errors["alg3.6_branch"] == "3.15"
    assert abs(errors["alg3.6"] / errors["equispaced"] - 1) <= 1e-3
    assert abs(errors["bopt"] / errors["equispaced"] - 1) <= 1e-3


def test_other_weights_do_worse(errors):
    assert errors["pcf_branch"] == "3.62" and errors["relaxed_branch"] == "3.63"
    for k in ("pcf", "relaxed", "one_over_n"):
        assert errors[k] >= 2.0 * errors["equispaced"], k
