"""Seeded synthetic inputs: node sets, sample vectors and Fourier coefficients.

This module holds no arithmetic of the NFFT or of the density-compensation
method. It only draws the node sets and random vectors that both the HIP path
and the CPU oracle consume, so that the two sides see identical inputs.

Node sets follow the grids of the paper's numerical section (Remark 5.1):
uniform random points, the jittered Cartesian grid, the polar grid with signed
radius (eq. (5.2)), the linogram grid (eq. (5.4)), plus an Archimedean spiral trajectory and plain
equispaced grids, and the band-limited test function of Example 5.5. All nodes are returned as float64 arrays of shape (N, d),
row-major, in the torus coordinates [-1/2, 1/2)^d.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "uniform_nodes",
    "jittered_nodes",
    "polar_nodes",
    "polar_area_weights",
    "linogram_nodes",
    "spiral_nodes",
    "equispaced_nodes",
    "triangle_pulse_coefficients",
    "triangle_pulse_samples",
    "complex_normal",
    "uniform_coefficients",
    "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _wrap(x: np.ndarray) -> np.ndarray:
    """Map coordinates onto [-1/2, 1/2) (the torus is 1-periodic)."""
    y = x - np.floor(x + 0.5)
    y[y >= 0.5] -= 1.0
    return y


def uniform_nodes(N: int, d: int, seed: int) -> np.ndarray:
    """Random grid of Remark 5.1(i): x = eta/2 with eta ~ U(-1, 1)^d."""
    g = rng(seed)
    return _wrap(0.5 * g.uniform(-1.0, 1.0, size=(N, d)))


def jittered_nodes(n: tuple[int, ...], seed: int, jitter: float = 0.25) -> np.ndarray:
    """Jittered Cartesian grid (Remark 5.1(i)).

    The printed formula of eq. (5.1) places the cell centres outside the torus
    for t = N_t and moves each point by up to a full cell. This generator uses
    the reading documented with the workloads: cell centres
    -1/2 + (t + 1/2)/n_t, t = 0..n_t-1, plus U(-jitter, jitter)/n_t per
    coordinate, wrapped onto [-1/2, 1/2).
    """
    g = rng(seed)
    axes = [(-0.5 + (np.arange(nt) + 0.5) / nt) for nt in n]
    mesh = np.meshgrid(*axes, indexing="ij")
    base = np.stack([a.reshape(-1) for a in mesh], axis=1)
    spacing = np.array([1.0 / nt for nt in n])
    pert = g.uniform(-jitter, jitter, size=base.shape) * spacing
    return _wrap(base + pert)


def polar_nodes(R: int, T: int) -> np.ndarray:
    """Polar grid with signed radius, eq. (5.2).

    r_j = j/R for j in I_R = {-R/2..R/2-1}, theta_t = pi t / T for t in I_T.
    Nodes are ordered angle-major (all radii of one ray are consecutive).
    All R*T nodes are kept, including the T duplicates at the origin; the
    single coordinate that lands on +1/2 is wrapped to -1/2.
    """
    j = np.arange(-R // 2, R // 2)
    t = np.arange(-T // 2, T // 2)
    r = j / R
    th = np.pi * t / T
    x1 = np.outer(np.cos(th), r).reshape(-1)
    x2 = np.outer(np.sin(th), r).reshape(-1)
    return _wrap(np.stack([x1, x2], axis=1))


def linogram_nodes(R: int, T: int) -> np.ndarray:
    """Linogram (pseudo-polar) grid of eq. (5.4): points on concentric squares,
    the set (j/R, (4t/T)(j/R)) and the set (-(4t/T)(j/R), j/R) for
    j = -R/2 .. R/2-1 and t = -T/4 .. T/4-1; N = R*T nodes (the T/2 + T/2
    points with j = 0 coincide at the origin). The Table 5.1 setting is
    R = 2M, T = 2R."""
    j = np.arange(-R // 2, R // 2, dtype=np.float64) / R
    t = 4.0 * np.arange(-T // 4, T // 4, dtype=np.float64) / T
    jj, tt = np.meshgrid(j, t, indexing="ij")
    bh = np.stack([jj.reshape(-1), (tt * jj).reshape(-1)], axis=1)
    bv = np.stack([-(tt * jj).reshape(-1), jj.reshape(-1)], axis=1)
    return _wrap(np.concatenate([bh, bv]))


def polar_area_weights(R: int, T: int) -> np.ndarray:
    """Geometric area weights for the polar grid of :func:`polar_nodes`.

    A substitute for the paper's weights on polar grids, where the weight
    system is rank deficient. Each node off the origin represents the annulus
    sector of area pi |r| / (R T) (ring spacing 1/R, 2T nodes per full circle);
    the disc of radius 1/(2R) around the origin is shared by its T duplicates.
    The weights are normalised to sum to one (exact quadrature of k = 0).
    Returned as complex128 with zero imaginary part, in the node order of
    :func:`polar_nodes`.
    """
    j = np.arange(-R // 2, R // 2)
    r = np.abs(j / R)
    w_r = np.where(j == 0, np.pi / (4.0 * R * R * T), np.pi * r / (R * T))
    w = np.tile(w_r, T)
    w = w / w.sum()
    return w.astype(np.complex128)


def spiral_nodes(N: int, M: int) -> np.ndarray:
    """Single Archimedean spiral trajectory with M/2 turns.

    t_j = j/N, r_j = t_j/2, theta_j = 2 pi (M/2) t_j, x_j = r_j (cos, sin).
    The spacing between neighbouring turns is 1/M.
    """
    t = np.arange(N) / N
    r = 0.5 * t
    th = 2.0 * np.pi * (M / 2) * t
    return _wrap(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))


def spiral_area_weights(N: int, M: int) -> np.ndarray:
    """Area weights for :func:`spiral_nodes`: proportional to the radius
    (arc-length times ring spacing), normalised to sum to one."""
    t = (np.arange(N) + 0.5) / N
    w = 0.5 * t
    w = w / w.sum()
    return w.astype(np.complex128)


def equispaced_nodes(n: int, d: int) -> np.ndarray:
    """Equispaced grid x_j = j/n, j in I_n^d (C-order, first index slowest)."""
    ax = np.arange(-n // 2, n // 2) / n
    mesh = np.meshgrid(*([ax] * d), indexing="ij")
    return np.stack([a.reshape(-1) for a in mesh], axis=1).astype(np.float64)


def triangle_pulse_coefficients(M: int, d: int, b: int) -> np.ndarray:
    """Example 5.5: fhat(v) = prod_t g(v_t) with the triangular pulse
    g(v) = (1 - |v / b|) on [-b, b] (zero outside), sampled at k in I_M
    (C order, k_t = -M/2 .. M/2 - 1), complex128."""
    k = np.arange(-M // 2, M // 2, dtype=np.float64)
    g = np.clip(1.0 - np.abs(k) / b, 0.0, None)
    out = g
    for _ in range(d - 1):
        out = np.multiply.outer(out, g)
    return out.reshape(-1).astype(np.complex128)


def triangle_pulse_samples(x: np.ndarray, b: int) -> np.ndarray:
    """Example 5.5: the inverse Fourier transform of the pulse above,
    f(x) = prod_t b sinc^2(b pi x_t) with sinc(t) = sin(t) / t, at the rows
    of x (a function on R^d, band-limited to [-b, b]^d), complex128."""
    x = np.asarray(x, dtype=np.float64)
    # numpy's sinc is sin(pi y) / (pi y)
    return np.prod(b * np.sinc(b * x) ** 2, axis=1).astype(np.complex128)


def complex_normal(shape, seed: int) -> np.ndarray:
    """complex128 array with i.i.d. N(0, 1) real and imaginary parts."""
    g = rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def uniform_coefficients(shape, seed: int, lo: float = 1.0, hi: float = 10.0) -> np.ndarray:
    """Real coefficients drawn from U[lo, hi] (the setting of Example 5.2),
    returned as complex128."""
    g = rng(seed)
    return g.uniform(lo, hi, size=shape).astype(np.complex128)


# Workload table. Each entry names its node generator and sizes; the weights
# recipe is described in words because the weights of the small case come
# from the paper's weight solver, which lives with the checker.
CONFIGS = {
    "C1": dict(d=2, M=32, N=4096, sigma=2.0, m=4, nodes="uniform", seed=1,
               weights="paper-scheme (least-squares on I_2M)", precision="f64"),
    "C2": dict(d=2, M=256, N=512 * 512, sigma=2.0, m=6, nodes="polar", R=512, T=512,
               weights="polar area weights", precision="f64|f32"),
    "C3": dict(d=3, M=64, N=128 * 64 * 64, sigma=2.0, m=4, nodes="jittered",
               n=(128, 64, 64), seed=4, weights="1/N", precision="f32"),
    "C4": dict(d=2, M=256, N=131072, sigma=2.0, m=6, nodes="spiral", nrhs=32,
               weights="spiral area weights", precision="f32"),
}


def make_nodes(cfg: dict) -> np.ndarray:
    kind = cfg["nodes"]
    if kind == "uniform":
        return uniform_nodes(cfg["N"], cfg["d"], cfg.get("seed", 1))
    if kind == "polar":
        return polar_nodes(cfg["R"], cfg["T"])
    if kind == "jittered":
        return jittered_nodes(tuple(cfg["n"]), cfg.get("seed", 4))
    if kind == "spiral":
        return spiral_nodes(cfg["N"], cfg["M"])
    raise ValueError(kind)
