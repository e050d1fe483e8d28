"""FP64 gridded variant of the moment images.  TEST INFRASTRUCTURE ONLY.

The paper computes each Chebyshev moment image by "a 2-D gridding operation
followed by an inverse FFT on the (r1, r2) grid" (§3.4) but names no gridding
kernel.  The kernel adopted is the exponential-of-semicircle (ES) function of
Barnett, Magland & af Klinteberg (SIAM J. Sci. Comput. 41, 2019),
``phi(z) = exp(beta (sqrt(1 - z^2) - 1))`` on ``|z| <= 1`` with support
``W = 8`` cells, ``beta = 2.30 W`` and a grid oversampled by ``sigma = 2``
(``M = 2N``); the grid correction divides by its Fourier transform
``psi(a) = (W/2) int_{-1}^{1} phi(z) cos(pi W z a / M) dz`` evaluated by
Gauss-Legendre quadrature.

Grid convention: sample q sits at ``X = M/2 - r1 M Delta``, ``Y = M/2 + r2 M Delta``
(so that grid signs follow the pixel convention); its taps are the W cells
starting at ``ceil(X - W/2)`` per axis, wrapped modulo M (the grid is periodic
with period ``1/Delta`` in r, the same period as the pixel-centre DFT);
``z = (cell - X) / (W/2)``.  The un-normalised inverse DFT with ``e^{+i}`` is
taken and the central ``N x N`` kept:
``I[a2][a1] = sum_{Y,X} G[Y][X] e^{i 2 pi ((X - M/2) a1 + (Y - M/2) a2)/M} / (psi(a1) psi(a2))``.
"""
from __future__ import annotations

import math

import numpy as np

ES_SUPPORT = 8
ES_BETA_PER_SUPPORT = 2.30
OVERSAMPLE = 2


def es_kernel(z, beta):
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) <= 1.0
    return np.where(inside, np.exp(beta * (np.sqrt(np.maximum(1.0 - z * z, 0.0)) - 1.0)), 0.0)


def es_correction(n_pix, M, W=ES_SUPPORT, beta=None, n_quad=128):
    """psi(a) for a = j - N/2, j = 0..N-1."""
    beta = ES_BETA_PER_SUPPORT * W if beta is None else beta
    z, wq = np.polynomial.legendre.leggauss(n_quad)
    a = np.arange(n_pix, dtype=np.float64) - n_pix / 2
    phi = es_kernel(z, beta)
    return (W / 2.0) * (np.cos(math.pi * W * np.outer(a, z) / M) @ (wq * phi))


def grid_coords(r1, r2, M, cell_deg):
    d = math.radians(cell_deg)
    return M / 2 - r1 * M * d, M / 2 + r2 * M * d


def grid_values(values, X, Y, M, W=ES_SUPPORT, beta=None):
    """Scatter complex ``values`` (P, Nq) onto P periodic M x M grids with the ES kernel."""
    beta = ES_BETA_PER_SUPPORT * W if beta is None else beta
    values = np.atleast_2d(values)
    P = values.shape[0]
    G = np.zeros((P, M, M), dtype=np.complex128)
    x0 = np.ceil(X - W / 2).astype(np.int64)
    y0 = np.ceil(Y - W / 2).astype(np.int64)
    for i in range(W):
        wx = es_kernel((x0 + i - X) / (W / 2), beta)
        cx = np.mod(x0 + i, M)
        for j in range(W):
            wy = es_kernel((y0 + j - Y) / (W / 2), beta)
            cy = np.mod(y0 + j, M)
            for p in range(P):
                np.add.at(G[p], (cy, cx), values[p] * (wx * wy))
    return G


def grid_to_image(G, n_pix, W=ES_SUPPORT, beta=None):
    """Corrected central N x N of the un-normalised inverse DFT of each grid."""
    P, M, _ = G.shape
    psi = es_correction(n_pix, M, W, beta)
    a = np.arange(n_pix) - n_pix // 2
    sign = np.where(a % 2 == 0, 1.0, -1.0)
    fac = (sign / psi)
    out = np.empty((P, n_pix, n_pix), dtype=np.complex128)
    idx = np.mod(a, M)
    for p in range(P):
        F = np.fft.ifft2(G[p]) * (M * M)
        out[p] = F[np.ix_(idx, idx)] * fac[:, None] * fac[None, :]
    return out


def gridded_moments(r, x, plan, n_pix, cell_deg, W=ES_SUPPORT):
    """The moment images M_{p,k} of §3.4 computed by ES gridding + inverse FFT; (n_slab, K, N, N)."""
    from .toi import slab_of, cheb_T
    M = OVERSAMPLE * n_pix
    p, s = slab_of(r[:, 2], plan)
    T = cheb_T(plan.K, s)
    X, Y = grid_coords(r[:, 0], r[:, 1], M, cell_deg)
    out = np.zeros((plan.n_slab, plan.K, n_pix, n_pix), dtype=np.complex128)
    for ps in range(plan.n_slab):
        sel = p == ps
        vals = (T[sel] * x[sel, None]).T
        out[ps] = grid_to_image(grid_values(vals, X[sel], Y[sel], M, W), n_pix, W)
    return out
