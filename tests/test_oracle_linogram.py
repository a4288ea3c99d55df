"""The linogram grid of eq. (5.4) and the Table 5.1 setting on the CPU.

* The generator against the definition, point by point (loops over j, t).
* Table 5.1's setting R = 2M, T = 2R has N = 8M^2 > |I_2M| = 4M^2, where the
  weights of Algorithm 3.6 reconstruct trigonometric polynomials of degree M
  exactly (Corollary 3.4): at M = 8 with the oracle's dense weights the
  error e_2 of (5.6) is at rounding level (the table prints 1.3e-15 there,
  for the phantom's coefficients; random coefficients stand in for them).
"""
import numpy as np

from oracle import ndft, weights, metrics
from paper_2302_00414_amd import workloads as wl


def test_linogram_nodes_follow_the_definition():
    R, T = 8, 16
    pts = []
    for j in range(-R // 2, R // 2):
        for t in range(-T // 4, T // 4):
            pts.append((j / R, 4 * t / T * j / R))      # x^BH
            pts.append((-4 * t / T * j / R, j / R))     # x^BV
    want = np.array(pts)
    want = want - np.floor(want + 0.5)                  # onto [-1/2, 1/2)
    got = wl.linogram_nodes(R, T)
    assert got.shape == (R * T, 2)
    key = lambda a: a[np.lexsort((a[:, 1], a[:, 0]))]
    assert np.array_equal(key(got), key(want))
    assert got.min() >= -0.5 and got.max() < 0.5


def test_table_5_1_setting_reconstructs_exactly():
    M = 8
    x = wl.linogram_nodes(2 * M, 4 * M)
    N = x.shape[0]
    assert N == 8 * M * M > (2 * M) ** 2
    w = weights.weights_lstsq(x, M)
    fh = wl.complex_normal(M * M, 140)
    f = ndft.forward(x, fh, M)
    e2 = metrics.rel_err(ndft.adjoint(x, w * f, M), fh)
    assert e2 <= 1e-13, e2
