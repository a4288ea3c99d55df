"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Small cases compare every output element with the step-by-step oracle NFFT
(O2, identical window) and with the exact sums (O1); full-size workloads
compare sampled outputs computed one by one from the exact sums.
Tolerances (relative l2 error): float64 path 1e-10, float32 path 1e-5; for
float64 against O2 only rounding separates the two, so 1e-12 is used there.
"""
import functools
import math

import numpy as np
import pytest
import torch

from oracle import ndft, nfft as onfft, metrics, window
from paper_2302_00414_amd import workloads as wl

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL_O2 = {"f64": 1e-12, "f32": 1e-5}
TOL_EXACT = {"f64": 1e-10, "f32": 1e-5}


def _plan(x, M, sigma, m, prec, max_rhs=1, tuning=None):
    from paper_2302_00414_amd.nfft import Plan
    print(f"[case] N={x.shape[0]} d={x.shape[1]} M={M} sigma={sigma} m={m} {prec} rhs={max_rhs} "
          f"tuning={tuning}", flush=True)
    return Plan(x, M, sigma, m, precision=prec, max_rhs=max_rhs, device="cuda:0", tuning=tuning)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


SMALL = [
    # d, M, sigma, m, N
    (1, 64, 2.0, 6, 900),
    (1, 1024, 2.0, 4, 5000),     # 8 tiles of 256
    (2, 32, 2.0, 4, 3000),       # 2 x 2 tiles
    (2, 48, 4.0 / 3.0, 5, 2500),  # M_sigma = 64, sigma != 2
    (2, 64, 2.0, 7, 7001),       # ragged N
    (2, 8, 2.0, 3, 50),          # single tile (16 <= 32), periodic self-neighbour
    (2, 32, 1.0, 4, 2000),       # sigma = 1: M_sigma = M, k = -M/2 at the edge of hat w's support
    (1, 64, 1.0, 3, 300),
    (3, 16, 2.0, 4, 4000),       # 4^3 tiles of 8
    (3, 8, 2.0, 2, 777),         # 2^3 tiles
]


def _what(M, sigma, m, d):
    """hat w on I_M in C order: the window's Fourier transform, by which the
    deconvolution D of (2.13) divides every output of the adjoint."""
    Ms = window.oversampled_size(M, sigma)
    h1 = window.phi_hat(np.arange(-M // 2, M // 2), m, sigma, Ms)
    W = h1
    for _ in range(d - 1):
        W = np.multiply.outer(W, h1)
    return W.ravel()


# Up to this ratio of the largest to the smallest hat w over I_M the
# deconvolution is well conditioned for the precision and outputs are also
# compared as they are. At sigma = 1 hat w reaches the edge of its support at
# |k| = M/2 (about 3e4 times below hat w(0) per dimension at m = 4): an output
# there carries that factor (to the power d at the corners) times the
# relative rounding of the grid sums, in any floating-point evaluation, the
# oracle's included. hat w * output, the spectrum before the division, is
# compared in every case.
KAPPA_PLAIN = {"f64": 1e4, "f32": 1e3}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,M,sigma,m,N", SMALL)
def test_adjoint_matches_oracle(d, M, sigma, m, N, prec):
    x = wl.uniform_nodes(N, d, 100 + N)
    w = (1.0 + 0.3 * wl.complex_normal(N, 101)) / N
    f = wl.complex_normal(N, 102)
    p = _plan(x, M, sigma, m, prec)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    ref = onfft.adjoint(x, w * f, M, sigma, m)
    W = _what(M, sigma, m, d)
    assert metrics.rel_err(W * got, W * ref) <= TOL_O2[prec]
    plain = W.max() / W.min() <= KAPPA_PLAIN[prec]
    if plain:
        assert metrics.rel_err(got, ref) <= TOL_O2[prec]
    S = np.ones_like(W) if plain else W
    if m >= 6 or prec == "f32":
        exact = ndft.adjoint(x, w * f, M)
        assert metrics.rel_err(S * got, S * exact) <= max(TOL_EXACT[prec],
                                                          2 * metrics.rel_err(S * ref, S * exact))
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,M,sigma,m,N", SMALL)
def test_forward_matches_oracle(d, M, sigma, m, N, prec):
    x = wl.uniform_nodes(N, d, 200 + N)
    fh = wl.complex_normal(M ** d, 201)
    W = _what(M, sigma, m, d)
    if W.max() / W.min() > KAPPA_PLAIN[prec]:
        # a spectrum shaped like hat w: D makes it white, so the window sums
        # are well conditioned (see KAPPA_PLAIN)
        fh = fh * (W / W.max())
    p = _plan(x, M, sigma, m, prec)
    got = _np(p.forward(torch.from_numpy(fh)))
    ref = onfft.forward(x, fh, M, sigma, m)
    assert metrics.rel_err(got, ref) <= TOL_O2[prec]
    p.close()


# the largest oversampled grid built, M_sigma = 4096 per dimension (d = 1, 2;
# the oracle's cost grows with the footprint, hence m = 2 for d = 2)
MAX_GRID = [
    # d, M, m, N
    (1, 2048, 8, 20000),
    (2, 2048, 2, 3000),
]


@functools.lru_cache(maxsize=None)
def _max_grid_case(d, M, m, N):
    x = wl.uniform_nodes(N, d, 400 + d)
    w = (1.0 + 0.3 * wl.complex_normal(N, 401)) / N
    f = wl.complex_normal(N, 402)
    fh = wl.complex_normal(M ** d, 403)
    return x, w, f, fh, onfft.adjoint(x, w * f, M, 2.0, m), onfft.forward(x, fh, M, 2.0, m)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,M,m,N", MAX_GRID)
def test_maximum_grid(d, M, m, N, prec):
    x, w, f, fh, ref_a, ref_f = _max_grid_case(d, M, m, N)
    p = _plan(x, M, 2.0, m, prec)
    assert p.info()["Ms"] == 4096
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    assert metrics.rel_err(got, ref_a) <= TOL_O2[prec]
    got_f = _np(p.forward(torch.from_numpy(fh)))
    assert metrics.rel_err(got_f, ref_f) <= TOL_O2[prec]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_edge_cases(prec):
    """Grid-aligned nodes (closed edge), duplicates in one cell, nodes at
    -1/2 and just below +1/2, coordinates outside the torus (wrapped), a
    crowded tile that splits into several work items, empty tiles."""
    M, sigma, m = 32, 2.0, 6
    Ms = window.oversampled_size(M, sigma)
    rng = np.random.default_rng(7)
    pts = [np.zeros((700, 2)),                                   # 700 duplicates at 0
           (rng.integers(-Ms // 2, Ms // 2, size=(300, 2)) / Ms),  # on grid points
           np.array([[-0.5, -0.5], [0.5 - 1e-17, 0.25], [0.4999999999, -0.5]]),
           rng.uniform(-3.0, 3.0, size=(200, 2)),                 # outside, wraps
           0.01 * rng.standard_normal((900, 2))]                  # crowded centre
    x = np.concatenate(pts)
    N = x.shape[0]
    w = (1.0 + 0.5 * wl.complex_normal(N, 8)) / N
    f = wl.complex_normal(N, 9)
    p = _plan(x, M, sigma, m, prec)
    info = p.info()
    assert info["items"] > info["tiles"] - 3
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    ref = onfft.adjoint(x, w * f, M, sigma, m)
    assert metrics.rel_err(got, ref) <= TOL_O2[prec]
    fh = wl.complex_normal(M * M, 10)
    got_f = _np(p.forward(torch.from_numpy(fh)))
    assert metrics.rel_err(got_f, onfft.forward(x, fh, M, sigma, m)) <= TOL_O2[prec]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_node_closed_form(prec):
    """P7 through the GPU: one node, f = 1, w = 1 gives h_k = exp(-2 pi i k.x)."""
    x = np.array([[0.123456789, -0.3141592653]])
    p = _plan(x, 16, 2.0, 6, prec)
    p.set_weights(np.ones(1))
    got = _np(p.adjoint(torch.ones(1, dtype=torch.complex128)))
    K = ndft.index_set(16, 2)
    assert metrics.rel_err(got, np.exp(-2j * math.pi * K @ x[0])) <= TOL_EXACT[prec]
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjointness_on_gpu(prec):
    """P6: <B F D fhat, g> = <fhat, D^* F^* B^* g> between the GPU forward
    and the GPU adjoint (unit weights)."""
    x = wl.uniform_nodes(5000, 2, 300)
    p = _plan(x, 64, 2.0, 5, prec)
    p.set_weights(np.ones(5000))
    fh = wl.complex_normal(64 * 64, 301)
    g = wl.complex_normal(5000, 302)
    a = _np(p.forward(torch.from_numpy(fh)))
    b = _np(p.adjoint(torch.from_numpy(g)))
    lhs, rhs = np.vdot(g, a), np.vdot(b, fh)
    assert abs(lhs - rhs) <= (1e-12 if prec == "f64" else 1e-5) * abs(lhs)
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_multi_rhs_equals_separate(prec):
    x = wl.uniform_nodes(3000, 2, 310)
    w = (1.0 + 0.2 * wl.complex_normal(3000, 311)) / 3000
    F = wl.complex_normal((5, 3000), 312)
    p = _plan(x, 32, 2.0, 6, prec, max_rhs=5)
    p.set_weights(w)
    both = _np(p.adjoint(torch.from_numpy(F)))
    ref = onfft.adjoint(x, w[None, :] * F, 32, 2.0, 6)
    for r in range(5):
        one = _np(p.adjoint(torch.from_numpy(F[r])))
        assert metrics.rel_err(both[r], one) <= (1e-14 if prec == "f64" else 1e-6)
        assert metrics.rel_err(both[r], ref[r]) <= TOL_O2[prec]
    fh = wl.complex_normal((5, 1024), 313)
    fb = _np(p.forward(torch.from_numpy(fh)))
    for r in range(5):
        assert metrics.rel_err(fb[r], _np(p.forward(torch.from_numpy(fh[r])))) <= 1e-14
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_multi_rhs_grouped_fft_lines(prec):
    """M = 256 (512-point lines) with 8 right-hand sides: the second FFT pass
    has 256 lines per right-hand side, so its first stage is radix 4, and the
    8 right-hand sides together group several lines per work-group. Every
    line is transformed as in a single call: the batched result equals the
    separate calls' (adjoint and forward)."""
    x = wl.uniform_nodes(20000, 2, 320)
    w = (1.0 + 0.2 * wl.complex_normal(20000, 321)) / 20000
    F = wl.complex_normal((8, 20000), 322)
    p = _plan(x, 256, 2.0, 6, prec, max_rhs=8)
    p.set_weights(w)
    both = _np(p.adjoint(torch.from_numpy(F)))
    for r in range(8):
        one = _np(p.adjoint(torch.from_numpy(F[r])))
        assert metrics.rel_err(both[r], one) <= (1e-14 if prec == "f64" else 1e-6)
    fh = wl.complex_normal((8, 256 * 256), 323)
    fb = _np(p.forward(torch.from_numpy(fh)))
    for r in range(8):
        assert metrics.rel_err(fb[r], _np(p.forward(torch.from_numpy(fh[r])))) <= 1e-14
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_node_permutation_invariance(prec):
    """P9: permuting the nodes (with their samples and weights) leaves the
    result unchanged up to rounding."""
    x = wl.uniform_nodes(4000, 2, 320)
    w = (1.0 + 0.2 * wl.complex_normal(4000, 321)) / 4000
    f = wl.complex_normal(4000, 322)
    perm = np.random.default_rng(5).permutation(4000)
    p1 = _plan(x, 32, 2.0, 6, prec)
    p1.set_weights(w)
    a = _np(p1.adjoint(torch.from_numpy(f)))
    p2 = _plan(x[perm], 32, 2.0, 6, prec)
    p2.set_weights(w[perm])
    b = _np(p2.adjoint(torch.from_numpy(f[perm])))
    assert metrics.rel_err(b, a) <= (1e-13 if prec == "f64" else 1e-6)
    p1.close()
    p2.close()


def test_state_and_argument_errors():
    from paper_2302_00414_amd import _lib
    from paper_2302_00414_amd.nfft import NfftError, Plan
    x = wl.uniform_nodes(100, 2, 330)
    p = _plan(x, 16, 2.0, 4, "f64", max_rhs=2)
    f = torch.zeros(100, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(NfftError) as e:
        p.adjoint(f)
    assert e.value.status == _lib.NFFT_ESTATE
    p.set_weights(np.ones(100))
    with pytest.raises(NfftError) as e:
        p.adjoint(torch.zeros((3, 100), dtype=torch.complex128, device="cuda:0"))
    assert e.value.status == _lib.NFFT_EINVAL
    bad = x.copy()
    bad[5, 1] = np.nan
    with pytest.raises(NfftError) as e:
        Plan(bad, 16, 2.0, 4, device="cuda:0")
    assert e.value.status == _lib.NFFT_EINVAL
    p.close()


# ------------------------------------------------------------ full workloads
def _sample_k(M, d, n, seed):
    K = ndft.index_set(M, d)
    rng = np.random.default_rng(seed)
    sel = rng.choice(K.shape[0], size=n, replace=False)
    corners = [0, K.shape[0] - 1, K.shape[0] // 2, K.shape[0] // 2 + M // 2]
    sel = np.unique(np.concatenate([sel, corners]))
    return sel, K[sel]


# "auto": the autotuned plan, the launch configuration the benchmark times
@pytest.mark.parametrize("tuning", [None, "auto", {"spread_mode": 5}, {"spread_mode": 7}])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_polar_512x512_M256(prec, tuning):
    """Polar grid R = T = 512 (N = 262144), M = 256, sigma = 2, m = 6, area
    weights: sampled outputs against the exact weighted sums."""
    R = T = 512
    x = wl.polar_nodes(R, T)
    w = wl.polar_area_weights(R, T)
    f = wl.complex_normal(x.shape[0], 3)
    p = _plan(x, 256, 2.0, 6, prec, tuning=tuning)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    sel, K = _sample_k(256, 2, 300, 11)
    exact = ndft.adjoint_at(x, w * f, K)
    assert metrics.rel_err(got[sel], exact) <= TOL_EXACT[prec]
    p.close()


@functools.lru_cache(maxsize=None)
def _c3_inputs():
    x = wl.jittered_nodes((128, 64, 64), 4)
    N = x.shape[0]
    w = np.full(N, 1.0 / N, dtype=np.complex128)
    f = wl.complex_normal(N, 5)
    print("[oracle] O2 adjoint of the jittered 128x64x64 set (about a minute)", flush=True)
    return x, w, f, onfft.adjoint(x, w * f, 64, 2.0, 4)


@pytest.mark.parametrize("tuning", [None, "auto", {"spread_mode": 7}])
def test_jittered_3d_M64(tuning):
    """Jittered 128 x 64 x 64 grid (N = 524288), d = 3, M = 64, m = 4, float32:
    the full output vector against the step-by-step oracle (O2), and sampled
    outputs against the exact sums."""
    x, w, f, ref = _c3_inputs()
    p = _plan(x, 64, 2.0, 4, "f32", tuning=tuning)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    e2 = metrics.rel_err(got, ref)
    sel, K = _sample_k(64, 3, 200, 12)
    exact = ndft.adjoint_at(x, w * f, K)
    e1 = metrics.rel_err(got[sel], exact)
    print(f"jittered 3-D f32: vs O2 (all {got.size} outputs) {e2:.3e}, vs exact sums (sampled) {e1:.3e}")
    assert e2 <= TOL_O2["f32"]
    assert e1 <= TOL_EXACT["f32"]
    p.close()


@functools.lru_cache(maxsize=None)
def _c4_inputs():
    N, M, nrhs = 131072, 256, 32
    x = wl.spiral_nodes(N, M)
    w = wl.spiral_area_weights(N, M)
    F = wl.complex_normal((nrhs, N), 6)
    print("[oracle] O2 adjoint of the 32 spiral right-hand sides", flush=True)
    return x, w, F, onfft.adjoint(x, w[None, :] * F, M, 2.0, 6)


@pytest.mark.parametrize("tuning", [None, "auto", {"spread_mode": 6}])
def test_spiral_32_rhs(tuning):
    """Archimedean spiral N = 131072, M = 256, m = 6, 32 right-hand sides in one
    float32 call: every right-hand side's full output vector against O2, and
    sampled outputs against the exact sums."""
    x, w, F, ref = _c4_inputs()
    M, nrhs = 256, F.shape[0]
    p = _plan(x, M, 2.0, 6, "f32", max_rhs=nrhs, tuning=tuning)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(F)))
    e2 = metrics.rel_err_rows(got, ref)
    sel, K = _sample_k(M, 2, 60, 13)
    exact = ndft.adjoint_at(x, w[None, :] * F, K)
    e1 = metrics.rel_err_rows(got[:, sel], exact)
    print(f"spiral 32 rhs f32: max over rhs vs O2 {e2.max():.3e}, vs exact sums (sampled) {e1.max():.3e}")
    assert e2.max() <= TOL_O2["f32"]
    assert e1.max() <= TOL_EXACT["f32"]
    p.close()


# ------------------------------------------------ the M = 32 correctness workloads
def _c1_weights():
    import os
    z = np.load(os.path.join(os.path.dirname(__file__), "golden", "c1_weights.npz"))
    return z["w_c1"], z["w_c1b"]


@pytest.mark.parametrize("tuning", [None, "auto"])
def test_c1_paper_weights_fp64(tuning):
    """d = 2, M = 32, N = 4096 uniform nodes (seed 1), m = 4, float64, samples
    of a random polynomial (f = A fhat by the exact sums), the oracle's
    Algorithm 3.6 weights (|I_2M| = N, minimum-norm solution of (3.15)): the
    reconstruction against the step-by-step oracle (O2) to 1e-10; the errors
    against the exact sums and against fhat are reported (the weights amplify
    the window error of m = 4 by about 1e5)."""
    x = wl.uniform_nodes(4096, 2, 1)
    fh = wl.complex_normal(32 * 32, 2)
    f = ndft.forward(x, fh, 32)
    w, _ = _c1_weights()
    p = _plan(x, 32, 2.0, 4, "f64", tuning=tuning)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    e2 = metrics.rel_err(got, onfft.adjoint(x, w * f, 32, 2.0, 4))
    e1 = metrics.rel_err(got, ndft.adjoint(x, w * f, 32))
    er = metrics.rel_err(got, fh)
    print(f"C1 f64: vs O2 {e2:.3e}, vs exact sums {e1:.3e}, vs fhat {er:.3e}")
    assert e2 <= 1e-10
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_c1b_example_5_2_size(prec):
    """d = 2, M = 32, N = 16384 uniform nodes (seed 7; the random-node size of
    Example 5.2, N_t = 128), coefficients from U[1, 10], m = 6, the oracle's
    Algorithm 3.6 weights (|I_2M| < N): the reconstruction against the exact
    sums (1e-10 / 1e-5) and against fhat itself (Corollary 3.4: exact up to
    the window error)."""
    x = wl.uniform_nodes(16384, 2, 7)
    fh = wl.uniform_coefficients(32 * 32, 8)
    f = ndft.forward(x, fh, 32)
    _, w = _c1_weights()
    p = _plan(x, 32, 2.0, 6, prec)
    p.set_weights(w)
    got = _np(p.adjoint(torch.from_numpy(f)))
    e1 = metrics.rel_err(got, ndft.adjoint(x, w * f, 32))
    er = metrics.rel_err(got, fh)
    print(f"C1b {prec}: vs exact sums {e1:.3e}, vs fhat {er:.3e}")
    assert e1 <= TOL_EXACT[prec]
    assert er <= TOL_EXACT[prec]
    p.close()
