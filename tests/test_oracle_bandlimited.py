"""Example 5.5 on the CPU: the band-limited test function and the comparison
of reconstructions, at a reduced size the oracle finishes in seconds.

* The input generator against the mathematics: the inverse Fourier transform
  of the triangular pulse g(v) = (1 - |v/b|) on [-b, b] is b sinc^2(b pi x)
  (quadrature at sample points), with the value b at x = 0, and the pulse
  samples at the frequencies k in I_M.
* The claims of Example 5.5, at M = 16, b = 6 on a jittered 36 x 36 grid
  (|I_2M| = 1024 <= N = 1296, the setting of the example): the weights of
  Algorithm 3.6 (dense least squares, oracle O3) and the optimized sparse
  matrix of Algorithm 4.3 reconstruct as well as an equispaced grid does
  (the truncation error of the integral dominates), while the PCF weights
  (3.62) and plain 1/N weights do clearly worse.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import ndft, weights as ow, bopt as ob
from paper_2302_00414_amd import workloads as wl


@pytest.mark.parametrize("b", [1, 6, 24])
@pytest.mark.parametrize("x", [0.0, 0.013, -0.07, 0.21, 0.5])
def test_pulse_samples_are_its_inverse_fourier_transform(b, x):
    # the pulse is even, so the transform is 2 * int_0^b (1 - v/b) cos(2 pi v x) dv
    # (QUADPACK's rule for cosine-weighted integrands)
    val, _ = integrate.quad(lambda v: 2.0 * (1.0 - v / b), 0.0, b, weight="cos",
                            wvar=2.0 * np.pi * x, limit=400, epsabs=1e-13, epsrel=1e-13)
    got = wl.triangle_pulse_samples(np.array([[x]]), b)[0]
    assert abs(got.imag) == 0.0
    assert abs(got.real - val) <= 1e-10 * b


def test_pulse_samples_tensor_product_and_peak():
    b = 24
    assert wl.triangle_pulse_samples(np.zeros((1, 2)), b)[0] == b * b
    x = np.array([[0.013, -0.21]])
    one = [wl.triangle_pulse_samples(x[:, [t]], b)[0] for t in range(2)]
    assert wl.triangle_pulse_samples(x, b)[0] == pytest.approx(one[0] * one[1], rel=1e-15)


def test_pulse_coefficients():
    M, b = 64, 24
    fh = wl.triangle_pulse_coefficients(M, 2, b).reshape(M, M)
    k = np.arange(-M // 2, M // 2)
    i0 = M // 2  # k = 0
    assert fh[i0, i0] == 1.0
    assert fh[i0, i0 + b // 2] == 0.5 and fh[i0 + b // 2, i0 - b // 2] == 0.25
    assert np.all(fh[np.abs(k) >= b, :] == 0) and np.all(fh[:, np.abs(k) >= b] == 0)
    assert np.all(fh.imag == 0) and fh.min() >= 0


def test_example_5_5_comparison_small():
    M, b, n = 16, 6, 36
    fh = wl.triangle_pulse_coefficients(M, 2, b)

    def err(h):
        return float(np.max(np.abs(h - fh)))

    xe = wl.equispaced_nodes(n, 2)
    e_eq = err(ndft.adjoint(xe, wl.triangle_pulse_samples(xe, b) / xe.shape[0], M))
    x = wl.jittered_nodes((n, n), 1, jitter=1.0)
    N = x.shape[0]
    assert (2 * M) ** 2 <= N
    f = wl.triangle_pulse_samples(x, b)
    e_w = err(ndft.adjoint(x, ow.weights_lstsq(x, M) * f, M))
    e_pcf = err(ndft.adjoint(x, ow.weights_pcf(x, M) * f, M))
    e_one = err(ndft.adjoint(x, f / N, M))
    B = ob.bopt(x, M, 2.0, 4)
    e_opt = err(ob.reconstruct(x, f, B, M, 2.0, 4))
    print(dict(equispaced=e_eq, alg36=e_w, bopt=e_opt, pcf=e_pcf, one_over_n=e_one))
    # the truncation error of the integral dominates: nothing beats the grid
    assert e_eq > 1e-2
    assert abs(e_w / e_eq - 1) <= 1e-3
    assert abs(e_opt / e_eq - 1) <= 1e-3
    assert e_pcf >= 1.3 * e_eq
    assert e_one >= 1.5 * e_eq
