"""O2: the NFFT and adjoint NFFT step by step (Algorithms 2.1 and 2.4).

    adjoint (Alg. 2.4):  g_l    = sum_j f_j w~_m(x_j - l/M_s),         l in I_Ms
                          ghat_k = |I_Ms|^-1 sum_l g_l e^{-2 pi i k.l/M_s}, k in I_M
                          h~_k   = ghat_k / hat w(k)
    forward (Alg. 2.1):  ghat_k = fhat_k / hat w(k) on I_M, 0 on I_Ms \\ I_M
                          g_l    = |I_Ms|^-1 sum_k ghat_k e^{+2 pi i k.l/M_s}
                          f~_j   = sum_{l in I_Ms,m(x_j)} g_l w~_m(x_j - l/M_s)

The window is the Kaiser-Bessel pair of :mod:`oracle.window`; w~_m is the
periodisation of the truncated window, so a grid index l is taken mod M_s and
every integer l with |M_s x_j - l| <= m contributes (the closed index set
(2.12)). The d-variate DFT of step 2 is numpy's FFT used as a library
routine. The weighted reconstruction (3.7) is ``adjoint(x, w * f, ...)``.

``dense_matrices`` builds D (2.13), F (2.14) and B (2.15) entry by entry for
tiny problems, so that the factorisations A ~ B F D and A^* ~ D^* F^* B^* can
be checked against the step-by-step code.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import window
from .ndft import freqs, index_set


def _wrap(x):
    y = x - np.floor(x + 0.5)
    return np.where(y >= 0.5, y - 1.0, y)


def _footprint(x, Ms, m, sigma):
    """Per dimension: the 2m+1 candidate integer grid indices l >= M_s x - m
    and the window values phi(M_s x - l) (zero outside |.| <= m)."""
    u = Ms * _wrap(np.atleast_2d(np.asarray(x, dtype=np.float64)))
    lo = np.ceil(u - m).astype(np.int64)
    offs = np.arange(2 * m + 1)
    ell = lo[:, :, None] + offs[None, None, :]            # (N, d, 2m+1)
    val = window.phi(u[:, :, None] - ell, m, sigma)       # (N, d, 2m+1)
    return ell, val


def spread(x, f, Ms, m, sigma):
    """Step 1 of Alg. 2.4: returns g on I_Ms stored at index l mod M_s,
    shape (R, Ms, ..., Ms)."""
    x = np.atleast_2d(x)
    N, d = x.shape
    F = np.asarray(f, dtype=np.complex128).reshape(-1, N)
    ell, val = _footprint(x, Ms, m, sigma)
    size = Ms ** d
    g = np.zeros((F.shape[0], size), dtype=np.complex128)
    offsets = list(itertools.product(range(2 * m + 1), repeat=d))
    # the (2m+1)^d footprint offsets go to one bincount in blocks (one call
    # per block and right-hand side instead of one per offset)
    nblk = max(1, min(len(offsets), (1 << 24) // max(N, 1)))
    for b0 in range(0, len(offsets), nblk):
        blk = offsets[b0:b0 + nblk]
        flat = np.zeros((len(blk), N), dtype=np.int64)
        wgt = np.ones((len(blk), N))
        for i, off in enumerate(blk):
            for t in range(d):
                flat[i] = flat[i] * Ms + np.mod(ell[:, t, off[t]], Ms)
                wgt[i] = wgt[i] * val[:, t, off[t]]
        flat = flat.reshape(-1)
        for r in range(F.shape[0]):
            c = (F[r][None, :] * wgt).reshape(-1)
            g[r] += np.bincount(flat, weights=c.real, minlength=size)
            g[r] += 1j * np.bincount(flat, weights=c.imag, minlength=size)
    return g.reshape((F.shape[0],) + (Ms,) * d)


def interpolate(x, g, Ms, m, sigma):
    """Step 3 of Alg. 2.1: f_j = sum_l g_l w~_m(x_j - l/M_s); g is
    (R, Ms, ..., Ms) stored at l mod M_s. Returns (R, N)."""
    x = np.atleast_2d(x)
    N, d = x.shape
    G = g.reshape(g.shape[0], -1)
    ell, val = _footprint(x, Ms, m, sigma)
    out = np.zeros((G.shape[0], N), dtype=np.complex128)
    for off in itertools.product(range(2 * m + 1), repeat=d):
        flat = np.zeros(N, dtype=np.int64)
        wgt = np.ones(N)
        for t in range(d):
            flat = flat * Ms + np.mod(ell[:, t, off[t]], Ms)
            wgt = wgt * val[:, t, off[t]]
        out += G[:, flat] * wgt
    return out


def _kidx(M, Ms, d):
    """Positions of k in I_M (C order) inside an FFT-ordered M_s^d array."""
    K = index_set(M, d)
    flat = np.zeros(K.shape[0], dtype=np.int64)
    for t in range(d):
        flat = flat * Ms + np.mod(K[:, t], Ms)
    return K, flat


def adjoint(x, f, M, sigma, m):
    """Algorithm 2.4: h~ ~ A^* f. ``f`` is (N,) or (R, N)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    Ms = window.oversampled_size(M, sigma)
    single = np.ndim(f) == 1
    g = spread(x, f, Ms, m, sigma)                                  # step 1
    axes = tuple(range(1, d + 1))
    ghat = np.fft.fftn(g, axes=axes).reshape(g.shape[0], -1) / Ms ** d  # step 2
    K, flat = _kidx(M, Ms, d)
    h = ghat[:, flat] / window.phi_hat_d(K, m, sigma, Ms)[None, :]  # step 3
    return h[0] if single else h


def forward(x, fhat, M, sigma, m):
    """Algorithm 2.1: f~ ~ A fhat. ``fhat`` is (M^d,) or (R, M^d)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    d = x.shape[1]
    Ms = window.oversampled_size(M, sigma)
    Fh = np.asarray(fhat, dtype=np.complex128)
    single = Fh.ndim == 1
    Fh = Fh.reshape(-1, M ** d)
    K, flat = _kidx(M, Ms, d)
    ghat = np.zeros((Fh.shape[0], Ms ** d), dtype=np.complex128)
    ghat[:, flat] = Fh / window.phi_hat_d(K, m, sigma, Ms)[None, :]   # step 1
    axes = tuple(range(1, d + 1))
    g = np.fft.ifftn(ghat.reshape((Fh.shape[0],) + (Ms,) * d), axes=axes)  # step 2
    out = interpolate(x, g, Ms, m, sigma)                           # step 3
    return out[0] if single else out


def dense_matrices(x, M, sigma, m):
    """D (2.13), F (2.14) and B (2.15) as dense arrays for tiny problems.

    Rows/columns of F and B over l in I_Ms and k in I_M are in C order with
    indices running from -M_s/2 (resp. -M/2); B sums the periodisation over
    all shifts z that reach the truncated support."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    N, d = x.shape
    Ms = window.oversampled_size(M, sigma)
    K = index_set(M, d)
    L = index_set(Ms, d)
    D = np.diag(1.0 / (Ms ** d * window.phi_hat_d(K, m, sigma, Ms)))
    F = np.exp(2j * math.pi * (L @ K.T) / Ms)
    zr = int(math.ceil((m + Ms) / Ms)) + 1
    B = np.zeros((N, L.shape[0]))
    for z in itertools.product(range(-zr, zr + 1), repeat=d):
        zz = np.array(z, dtype=np.float64)
        for j in range(N):
            tt = Ms * (x[j][None, :] + zz[None, :]) - L
            B[j] += np.prod(window.phi(tt, m, sigma), axis=1)
    return D, F, B

