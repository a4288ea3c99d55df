"""O5: weighted iterative refinement of the density-compensation
reconstruction. Test infrastructure: only the tests, the smoke check and the
CPU baseline of the benchmark use this package.

With weights W = diag(w) from Algorithm 3.6, the matrix A^* W A equals
I + E with the Toeplitz matrix E = (eps_{l-k}) of the residuals (3.36), and
the proof of Theorem 3.15 writes its inverse as the Neumann series
sum_n (I - A^* W A)^n, which converges when ||E||_2 < 1. The paper remarks
that W can be used in an iterative procedure to improve the reconstruction
A^* W f of Algorithm 3.7 without stating one. The one taken here is the
plain iteration whose iterates are the partial sums of that series applied
to A^* W f:

    fhat_0     = A^* W f                           (Algorithm 3.7, eq. (3.7))
    fhat_{k+1} = fhat_k + A^* W (f - A fhat_k),    k = 0, 1, ...

so fhat_k = sum_{n=0}^{k} (I - A^* W A)^n A^* W f, which tends to the
weighted least-squares solution (A^* W A)^{-1} A^* W f; for samples of a
trigonometric polynomial of degree M (f = A fhat) its error is
fhat - fhat_k = (I - A^* W A)^{k+1} fhat, of 2-norm at most
(|I_M| eps)^{k+1} ||fhat||_2 by the bound ||E||_2 <= |I_M| eps used for (3.37).

The products with A and A^* are exact sums (O1, ``op="ndft"``) or the
reference NFFT of Algorithms 2.1 and 2.4 (O2, ``op="nfft"``).
"""
from __future__ import annotations

import numpy as np

from . import ndft, nfft


def _ops(x, M, op, sigma, m):
    if op == "ndft":
        return (lambda fh: ndft.forward(x, fh, M)), (lambda f: ndft.adjoint(x, f, M))
    if op == "nfft":
        return (lambda fh: nfft.forward(x, fh, M, sigma, m)), (lambda f: nfft.adjoint(x, f, M, sigma, m))
    raise ValueError(op)


def refine(x, f, w, M, iters, op="ndft", sigma=2.0, m=8):
    """fhat_iters of the iteration above and the relative residuals
    ||f - A fhat_k||_2 / ||f||_2, k = 0..iters (over all right-hand sides).
    ``f`` is (N,) or (R, N); ``w`` is (N,)."""
    fwd, adj = _ops(np.atleast_2d(np.asarray(x, dtype=np.float64)), M, op, sigma, m)
    f = np.asarray(f, dtype=np.complex128)
    w = np.asarray(w, dtype=np.complex128)
    fn = np.linalg.norm(f)
    fhat = adj(w * f)                  # fhat_0, the direct reconstruction
    res = []
    for k in range(iters + 1):
        r = f - fwd(fhat)              # residual of fhat_k
        res.append(np.linalg.norm(r) / fn if fn > 0 else 0.0)
        if k == iters:
            break
        fhat = fhat + adj(w * r)       # fhat_{k+1}
    return fhat, np.array(res)
