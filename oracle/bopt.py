"""O4: the optimized sparse matrix B_opt (Algorithm 4.3) and the
reconstruction h_opt = D^* F^* B_opt^* f (Algorithm 4.4, eq. (4.12)).

Test infrastructure: plain numpy in float64, shares nothing with the HIP
path.

Grid columns l run over I_Ms in C order with indices from -M_s/2, as in
``oracle.nfft.dense_matrices``. Per column:

* the index set of (4.15): the nodes j whose closed window support reaches
  l periodically, |M_s x_j - l + M_s z| <= m for some integer vector z (the
  nonzero pattern of column l of B; the printed condition adds z without the
  factor M_s, which would admit every node);
* G_l = H_l^* H_l by the Dirichlet-kernel product (4.13), with
  H_l = (e^{-2 pi i k.x_j})_{k in I_M, j in the set} of (4.11);
* v_l = |I_Ms|^{-1} H_l^* D^{-1} f_l by (4.14),
  v_j = sum_{k in I_M} w^(k) e^{2 pi i k.(x_j - l/M_s)};
* b_l minimises ||H_l b - |I_Ms|^{-1} D^{-1} f_l||_2 over real b (B_opt is
  declared real while (4.12)'s formula is complex): the real normal
  equations Re(G_l) b = Re(v_l), solved in the minimum-norm least-squares
  sense (numpy lstsq), which also covers rank-deficient columns (duplicate
  nodes).

``bopt_dense`` solves the same column problems from the definition (the
stacked real least-squares problem with H_l built entry by entry) for tiny
inputs; ``objective`` evaluates the Frobenius objective (4.9) column by column.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import window
from .ndft import index_set


def _wrap(x):
    y = x - np.floor(x + 0.5)
    return np.where(y >= 0.5, y - 1.0, y)


def column_sets(x, M, sigma, m):
    """CSR (indptr, nodes) of the index sets (4.15) over l in I_Ms (C order,
    from -M_s/2). Nodes of a column in increasing order."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    u = Ms * _wrap(x)
    lo = np.ceil(u - m).astype(np.int64)
    rows, cols = [], []
    offs = np.arange(2 * m + 1)
    import itertools
    for off in itertools.product(offs, repeat=d):
        ell = lo + np.array(off)[None, :]                       # (N, d)
        ok = np.all(np.abs(u - ell) <= m, axis=1)
        # column index in C order of I_Ms (indices from -M_s/2, periodic)
        c = np.zeros(N, dtype=np.int64)
        for t in range(d):
            c = c * Ms + np.mod(ell[:, t] + Ms // 2, Ms)
        rows.append(np.nonzero(ok)[0])
        cols.append(c[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    # a node reaches a cell at most once (the footprint spans 2m+1 < M_s cells)
    mat = sp.csr_matrix((np.ones(len(rows)), (cols, rows)), shape=(Ms ** d, N))
    mat.sort_indices()
    return mat.indptr.copy(), mat.indices.copy()


def gram(xs, M):
    """(4.13): [H^* H]_{h,j} = prod_t (D_{M/2-1}(x_ht - x_jt) + e^{-M pi i (x_ht - x_jt)}),
    D_{M/2-1}(s) = sin((M-1) pi s) / sin(pi s) (value M - 1 at integers)."""
    xs = np.atleast_2d(xs)
    G = np.ones((xs.shape[0], xs.shape[0]), dtype=np.complex128)
    for t in range(xs.shape[1]):
        s = xs[:, t][:, None] - xs[:, t][None, :]
        den = np.sin(math.pi * s)
        small = np.abs(den) < 1e-300
        dk = np.where(small, 0.0, np.sin((M - 1) * math.pi * s) / np.where(small, 1.0, den))
        # at integer s the Dirichlet kernel is (M - 1) cos((M - 1) pi s) / cos(pi s) = +-(M - 1)
        dk = np.where(small, (M - 1) * np.cos((M - 1) * math.pi * s) / np.cos(math.pi * s), dk)
        G = G * (dk + np.exp(-1j * M * math.pi * s))
    return G


def rhs(xs, l, M, sigma, m):
    """(4.14): v_j = sum_{k in I_M} w^(k) e^{2 pi i k.(x_j - l/M_s)}, the
    transform w^ of the window (ŵ = phi_hat, so |I_Ms|^{-1} D^{-1} = diag ŵ);
    evaluated as a product of one-dimensional sums."""
    xs = np.atleast_2d(xs)
    Ms = window.oversampled_size(M, sigma)
    k = np.arange(-M // 2, M // 2)
    wh = window.phi_hat(k, m, sigma, Ms)
    v = np.ones(xs.shape[0], dtype=np.complex128)
    for t in range(xs.shape[1]):
        s = xs[:, t] - l[t] / Ms
        v = v * (np.exp(2j * math.pi * np.outer(s, k)) @ wh)
    return v


def _grid_index(c, Ms, d):
    """C-order column number -> centred grid index l in I_Ms."""
    l = np.zeros(d, dtype=np.int64)
    for t in range(d - 1, -1, -1):
        l[t] = c % Ms - Ms // 2
        c //= Ms
    return l


def _solve_column(xw, js, c, M, sigma, m, rcond):
    """Values of column c (nodes js): the real normal equations of (4.12),
    Re(H^* H) b = Re(v), by a minimum-norm least-squares solve."""
    Ms = window.oversampled_size(M, sigma)
    l = _grid_index(c, Ms, xw.shape[1])
    G = gram(xw[js], M)
    v = rhs(xw[js], l, M, sigma, m)
    b, *_ = np.linalg.lstsq(G.real, v.real, rcond=rcond)
    return b


def bopt(x, M, sigma, m, rcond=1e-13):
    """Algorithm 4.3. Returns B_opt as a scipy CSR matrix N x |I_Ms| (real)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    indptr, nodes = column_sets(x, M, sigma, m)
    xw = _wrap(x)
    vals = np.zeros(len(nodes))
    for c in range(Ms ** d):
        s, e = indptr[c], indptr[c + 1]
        if s == e:
            continue
        vals[s:e] = _solve_column(xw, nodes[s:e], c, M, sigma, m, rcond)
    # stored by columns: transpose of CSC
    return sp.csc_matrix((vals, nodes, indptr), shape=(N, Ms ** d)).tocsr()


def bopt_columns(x, M, sigma, m, cols, rcond=1e-13):
    """The columns `cols` of Algorithm 4.3 alone: {c: (nodes, values)}, nodes
    in increasing order (for checking single columns of large problems)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    indptr, nodes = column_sets(x, M, sigma, m)
    xw = _wrap(x)
    out = {}
    for c in cols:
        js = nodes[indptr[c]:indptr[c + 1]]
        out[int(c)] = (js, _solve_column(xw, js, c, M, sigma, m, rcond) if len(js) else np.zeros(0))
    return out


def bopt_dense(x, M, sigma, m):
    """The column problems of (4.10) from the definition: H_l entry by entry,
    real least squares of the stacked [Re; Im] system. Tiny inputs only."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    K = index_set(M, d)
    L = index_set(Ms, d)
    wh = window.phi_hat_d(K, m, sigma, Ms)
    indptr, nodes = column_sets(x, M, sigma, m)
    B = np.zeros((N, Ms ** d))
    for c in range(Ms ** d):
        js = nodes[indptr[c]:indptr[c + 1]]
        if len(js) == 0:
            continue
        H = np.exp(-2j * math.pi * (K @ x[js].T))                 # (4.11)
        r = wh * np.exp(-2j * math.pi * (K @ L[c]) / Ms)           # |I_Ms|^-1 D^-1 f_l
        A = np.vstack([H.real, H.imag])
        y = np.concatenate([r.real, r.imag])
        b, *_ = np.linalg.lstsq(A, y, rcond=None)
        B[js, c] = b
    return B


def objective(x, B, M, sigma, m):
    """|| A^* B - |I_Ms|^{-1} D^{-1} F^* ||_F^2 of (4.9) (dense, tiny inputs)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    K = index_set(M, d)
    L = index_set(Ms, d)
    Astar = np.exp(-2j * math.pi * (K @ x.T))
    wh = window.phi_hat_d(K, m, sigma, Ms)
    target = wh[:, None] * np.exp(-2j * math.pi * (K @ L.T) / Ms)
    Bd = B.toarray() if sp.issparse(B) else B
    return float(np.linalg.norm(Astar @ Bd - target) ** 2)


def reconstruct(x, f, B, M, sigma, m):
    """Algorithm 4.4 step 1: h_opt = D^* F^* B_opt^* f (B_opt real, so
    B^* = B^T): the grid g = B^T f over I_Ms, then the d-variate DFT and
    the deconvolution of Algorithm 2.4 steps 2 and 3."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    F = np.asarray(f, dtype=np.complex128).reshape(-1, N)
    g = (B.T @ F.T).T                                           # (R, Ms^d), C order from -Ms/2
    g = g.reshape((F.shape[0],) + (Ms,) * d)
    # centred C order -> storage at l mod M_s (index l + Ms/2 -> l mod Ms)
    g = np.fft.ifftshift(g, axes=tuple(range(1, d + 1)))
    ghat = np.fft.fftn(g, axes=tuple(range(1, d + 1))).reshape(F.shape[0], -1) / Ms ** d
    K = index_set(M, d)
    flat = np.zeros(K.shape[0], dtype=np.int64)
    for t in range(d):
        flat = flat * Ms + np.mod(K[:, t], Ms)
    h = ghat[:, flat] / window.phi_hat_d(K, m, sigma, Ms)[None, :]
    return h[0] if np.ndim(f) == 1 else h


def inverse_adjoint(x, h, B, M, sigma, m):
    """Remark 4.6: an approximate solution of A^* f = h (the inverse adjoint
    NFFT), f = B_opt F D h: Algorithm 2.1 steps 1 and 2 (deconvolution, zero
    padding, inverse DFT) followed by B_opt in place of the window matrix B."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    H = np.asarray(h, dtype=np.complex128).reshape(-1, M ** d)
    K = index_set(M, d)
    flat = np.zeros(K.shape[0], dtype=np.int64)
    for t in range(d):
        flat = flat * Ms + np.mod(K[:, t], Ms)
    ghat = np.zeros((H.shape[0], Ms ** d), dtype=np.complex128)
    ghat[:, flat] = H / window.phi_hat_d(K, m, sigma, Ms)[None, :]
    g = np.fft.ifftn(ghat.reshape((H.shape[0],) + (Ms,) * d), axes=tuple(range(1, d + 1)))
    # storage at l mod M_s -> centred C order (index l + M_s/2)
    g = np.fft.fftshift(g, axes=tuple(range(1, d + 1))).reshape(H.shape[0], -1)
    f = (B @ g.T).T
    return f[0] if np.ndim(h) == 1 else f
