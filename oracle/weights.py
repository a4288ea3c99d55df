"""O3: density-compensation factors of Algorithm 3.6.

The augmented quadrature conditions (3.14) read A_2M^T w = e_0 on I_2M, with
A_2M the nonequispaced Fourier matrix (2.7) of size N x (2M)^d and e_0 the
unit vector of k = 0. Algorithm 3.6 branches on |I_2M| = (2M)^d versus N:

* |I_2M| <= N (underdetermined, Sec. 3.1.1): the minimum-norm solution via the
  normal equations of the second kind (3.15),
      A_2M^T conj(A_2M) v = e_0,   w = conj(A_2M) v;
* |I_2M| >  N (overdetermined, Sec. 3.1.2): the least-squares solution via the
  normal equations of the first kind (3.16),
      conj(A_2M) A_2M^T w = conj(A_2M) e_0 = 1_N.

``weights_cg`` follows the algorithm with the conjugate-gradient method on
these Hermitian positive semi-definite systems (x_0 = 0; the paper does not
fix tolerance or iteration count). The products with A_2M^T and conj(A_2M)
are adjoint / forward transforms at size 2M: exact sums (O1) or the NFFT (O2).

``weights_lstsq`` computes the same minimum-norm least-squares solution of
A_2M^T w = e_0 with a dense LAPACK solve; it covers both branches and is the
reference for small problems.

``residual`` is epsilon = max_k |[A_2M^T w]_k - delta_{0,k}| over I_2M, the
quantity of (3.36) that enters the bounds (3.37) and (3.46).

Two weight choices from the literature that Section 3.4 compares with:
``weights_pcf`` (3.62), the minimiser of the Frobenius problem (3.61), and
``weights_relaxed``, the solution of the summed conditions A A^* w = 1_N
(3.63), both from the dense A A^* of (3.60).
"""
from __future__ import annotations

import numpy as np

from . import ndft, nfft
from .ndft import fourier_matrix, index_set


def _e0(M2: int, d: int) -> np.ndarray:
    K = index_set(M2, d)
    return np.all(K == 0, axis=1).astype(np.complex128)


def weights_lstsq(x: np.ndarray, M: int) -> np.ndarray:
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    A2 = fourier_matrix(x, 2 * M)
    w, *_ = np.linalg.lstsq(A2.T, _e0(2 * M, x.shape[1]), rcond=None)
    return w


def _ops(x, M2, matvec, sigma, m):
    """Return (AT, Abar): y -> A_2M^T y and v -> conj(A_2M) v."""
    if matvec == "ndft":
        adj = lambda c: ndft.adjoint(x, c, M2)
        fwd = lambda v: ndft.forward(x, v, M2)
    elif matvec == "nfft":
        adj = lambda c: nfft.adjoint(x, c, M2, sigma, m)
        fwd = lambda v: nfft.forward(x, v, M2, sigma, m)
    else:
        raise ValueError(matvec)
    AT = lambda y: np.conj(adj(np.conj(y)))
    Abar = lambda v: np.conj(fwd(np.conj(v)))
    return AT, Abar


def cg(apply, b, tol=1e-13, maxit=1000):
    """Conjugate gradients for a Hermitian positive (semi-)definite operator,
    starting from zero. Returns (solution, iterations, final relative residual)."""
    xk = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    nb = np.sqrt(np.vdot(b, b).real)
    it = 0
    while it < maxit and np.sqrt(rr) > tol * nb:
        Ap = apply(p)
        alpha = rr / np.vdot(p, Ap).real
        xk = xk + alpha * p
        r = r - alpha * Ap
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return xk, it, float(np.sqrt(rr) / nb)


def weights_cg(x, M, matvec="ndft", sigma=2.0, m=8, tol=1e-13, maxit=1000):
    """Algorithm 3.6 with CG. Returns (w, info dict)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    M2 = 2 * M
    AT, Abar = _ops(x, M2, matvec, sigma, m)
    if M2 ** d <= N:                     # step 2, first branch: (3.15)
        e0 = _e0(M2, d)
        v, it, rel = cg(lambda y: AT(Abar(y)), e0, tol, maxit)
        w = Abar(v)
        branch = "3.15"
    else:                                # step 2, second branch: (3.16)
        ones = np.ones(N, dtype=np.complex128)
        w, it, rel = cg(lambda y: Abar(AT(y)), ones, tol, maxit)
        branch = "3.16"
    return w, dict(iterations=it, rel_residual=rel, branch=branch)


def residual(x, w, M) -> float:
    """epsilon = ||A_2M^T w - e_0||_inf over I_2M (complex moduli)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    M2 = 2 * M
    r = np.conj(ndft.adjoint(x, np.conj(w), M2)) - _e0(M2, x.shape[1])
    return float(np.max(np.abs(r)))


# ------------------------------------------------ weights from the literature
def gram_nodes(x, M) -> np.ndarray:
    """[A A^*]_{j,h} = sum_{k in I_M} e^{2 pi i k.(x_j - x_h)} (3.60), from the
    Fourier matrix (2.7) itself (dense, small N)."""
    A = fourier_matrix(np.atleast_2d(np.asarray(x, dtype=np.float64)), M)
    return A @ A.conj().T


def weights_pcf(x, M) -> np.ndarray:
    """(3.62): the minimiser of ||A A^* W - I_N||_F over diagonal W,
    w_j = |I_M| / sum_h |[A A^*]_{j,h}|^2."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    H = gram_nodes(x, M)
    return (M ** x.shape[1]) / np.sum(np.abs(H) ** 2, axis=1) + 0j


def weights_relaxed(x, M) -> np.ndarray:
    """(3.63): A A^* w = 1_N, the minimum-norm least-squares solution (dense)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    H = gram_nodes(x, M)
    w, *_ = np.linalg.lstsq(H, np.ones(x.shape[0], dtype=np.complex128), rcond=None)
    return w
