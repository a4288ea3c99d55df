"""O1: the nonequispaced discrete Fourier transform by its definition.

    forward (2.5):  f_j = sum_{k in I_M} fhat_k exp(+2 pi i k.x_j),  j = 1..N
    adjoint (2.6):  h_k = sum_{j=1}^N  f_j   exp(-2 pi i k.x_j),  k in I_M

i.e. f = A fhat and h = A^* f with the nonequispaced Fourier matrix A of (2.7).
The weighted adjoint of (3.6)/(3.7), h^w = A^* W f, is ``adjoint(x, w * f)``.

I_M = {-M/2, ..., M/2-1}^d is enumerated in C order (k_1 slowest). Phase
tables exp(2 pi i k_t x_{j,t}) are evaluated entry by entry in float64 (no
angle recurrences); the d-variate sums are contracted with plain matrix
products over chunks of nodes. ``adjoint_loops`` / ``forward_loops`` are the
same sums as pure-Python loops for tiny inputs.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def freqs(M: int) -> np.ndarray:
    """The 1-D index set I_M = {-M/2, ..., M/2 - 1}."""
    if M % 2:
        raise ValueError("M must be even")
    return np.arange(-M // 2, M // 2)


def index_set(M: int, d: int) -> np.ndarray:
    """All k in I_M^d as a (M^d, d) integer array, C order."""
    ax = freqs(M)
    mesh = np.meshgrid(*([ax] * d), indexing="ij")
    return np.stack([a.reshape(-1) for a in mesh], axis=1)


def fourier_matrix(x: np.ndarray, M: int) -> np.ndarray:
    """A = (exp(2 pi i k.x_j))_{j, k} in C^{N x M^d}, eq. (2.7)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    K = index_set(M, x.shape[1])
    return np.exp(1j * TWO_PI * (x @ K.T.astype(np.float64)))


def _phase_tables(x: np.ndarray, M: int):
    k = freqs(M).astype(np.float64)
    return [np.exp(1j * TWO_PI * np.outer(x[:, t], k)) for t in range(x.shape[1])]


def _khatri_rao(tabs):
    """Row-wise Kronecker product of (J, M) tables -> (J, M^len(tabs))."""
    out = tabs[0]
    for t in tabs[1:]:
        out = (out[:, :, None] * t[:, None, :]).reshape(out.shape[0], -1)
    return out


def _chunk(M: int, d: int) -> int:
    inner = M ** (d - 1)
    return int(max(256, min(1 << 16, (1 << 23) // max(inner, 1))))


def adjoint(x: np.ndarray, f: np.ndarray, M: int) -> np.ndarray:
    """h = A^* f. ``f`` is (N,) or (R, N); returns (M^d,) or (R, M^d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    F = f.reshape(1, N) if single else f
    R = F.shape[0]
    h = np.zeros((R, M, M ** (d - 1)), dtype=np.complex128)
    J = _chunk(M, d)
    for s in range(0, N, J):
        xs = x[s:s + J]
        tabs = [np.conj(t) for t in _phase_tables(xs, M)]
        rest = _khatri_rao(tabs[1:]) if d > 1 else np.ones((xs.shape[0], 1), np.complex128)
        for r in range(R):
            h[r] += (tabs[0] * F[r, s:s + J, None]).T @ rest
    h = h.reshape(R, M ** d)
    return h[0] if single else h


def forward(x: np.ndarray, fhat: np.ndarray, M: int) -> np.ndarray:
    """f = A fhat. ``fhat`` is (M^d,) or (R, M^d); returns (N,) or (R, N)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    fh = np.asarray(fhat, dtype=np.complex128)
    single = fh.ndim == 1
    Fh = fh.reshape(1, -1) if single else fh
    R = Fh.shape[0]
    out = np.zeros((R, N), dtype=np.complex128)
    J = _chunk(M, d)
    for s in range(0, N, J):
        xs = x[s:s + J]
        tabs = _phase_tables(xs, M)
        rest = _khatri_rao(tabs[1:]) if d > 1 else np.ones((xs.shape[0], 1), np.complex128)
        for r in range(R):
            part = tabs[0] @ Fh[r].reshape(M, M ** (d - 1))
            out[r, s:s + J] = np.sum(part * rest, axis=1)
    return out[0] if single else out


def adjoint_at(x: np.ndarray, f: np.ndarray, kvec: np.ndarray) -> np.ndarray:
    """h_k = sum_j f_j exp(-2 pi i k.x_j) for selected frequencies only.

    ``kvec`` is (K, d) integer; ``f`` is (N,) or (R, N). Used to check single
    outputs of large transforms one by one.
    """
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 1
    F = f.reshape(1, -1) if single else f
    K = np.asarray(kvec, dtype=np.float64).reshape(-1, x.shape[1])
    out = np.zeros((F.shape[0], K.shape[0]), dtype=np.complex128)
    J = 1 << 15
    for s in range(0, x.shape[0], J):
        E = np.exp(-1j * TWO_PI * (x[s:s + J] @ K.T))
        out += F[:, s:s + J] @ E
    return out[0] if single else out


def forward_at(x: np.ndarray, fhat: np.ndarray, M: int, rows) -> np.ndarray:
    """f_j of the forward sum for the node indices ``rows`` only."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return forward(x[np.asarray(rows)], fhat, M)


def adjoint_loops(x, f, M):
    """Pure-Python triple loop of (2.6); tiny inputs only."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    out = []
    for k in itertools.product(range(-M // 2, M // 2), repeat=d):
        s = 0j
        for j in range(N):
            ang = 0.0
            for t in range(d):
                ang += k[t] * x[j, t]
            s += f[j] * complex(math.cos(TWO_PI * ang), -math.sin(TWO_PI * ang))
        out.append(s)
    return np.array(out)


def forward_loops(x, fhat, M):
    """Pure-Python loops of (2.5); tiny inputs only."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    ks = list(itertools.product(range(-M // 2, M // 2), repeat=d))
    out = []
    for j in range(N):
        s = 0j
        for i, k in enumerate(ks):
            ang = sum(k[t] * x[j, t] for t in range(d))
            s += fhat[i] * complex(math.cos(TWO_PI * ang), math.sin(TWO_PI * ang))
        out.append(s)
    return np.array(out)
