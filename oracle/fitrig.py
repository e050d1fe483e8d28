"""FP64 CPU oracle of the FITrig stage fed by TOI.  TEST INFRASTRUCTURE ONLY.

The paper states what FITrig computes but not its formulas:
  * tLISI compares one tile between two adjacent difference images built from
    the three youngest snapshots; it lies in [0, 1], 1 meaning identical and
    low values flagging a transient (tile 32 x 32);
  * after the run, a Fourier transform along time of the tLISI cube, harmonic
    summing of the power spectrum, a significance map, a 5-sigma threshold and
    merging of connected significant tiles into bounding boxes in full
    resolution pixels; a non-periodic variant thresholds sum_t (1 - tLISI) at
    4 sigma.

The published tLISI formula (FITrig paper) is not available here, so tLISI is
a stand-in with every property above (parity with FITrig itself is unpinned):
``X = I_{t-1} - I_{t-2}``, ``Y = I_t - I_{t-1}``; ``L`` is the range of the
pair; per tile the SSIM form of Wang et al. (IEEE TIP 13, 2004) with
``C1 = (0.01 L)^2``, ``C2 = (0.03 L)^2`` and population statistics gives S and
``tLISI = clamp((1 + S) / 2, 0, 1)`` (1 everywhere when ``L = 0``).

Detection runs over a sliding window of the 16 newest tLISI maps (the
streaming reading) or over the whole run's cube of L maps (the paper's
after-the-run statistic): per tile the DFT power of the mean-removed series at
f = 1..L/2, harmonic sums over h in {1, 2, 4, 8} harmonics normalised by sqrt(h),
the non-periodic sum of (1 - tLISI), z-scores over all tiles with the
population standard deviation, thresholds 5 (periodic) or 4 (non-periodic),
8-connected components of the flagged tiles and one box per component.
"""
from __future__ import annotations

import math

import numpy as np

WINDOW = 16
HARMONICS = (1, 2, 4, 8)


def tlisi(img_tm2, img_tm1, img_t, tile=32):
    """One tLISI map of shape (N // tile, N // tile) from the three youngest images."""
    a = np.asarray(img_tm2, dtype=np.float64)
    b = np.asarray(img_tm1, dtype=np.float64)
    c = np.asarray(img_t, dtype=np.float64)
    X = b - a
    Y = c - b
    ny, nx = X.shape[0] // tile, X.shape[1] // tile
    L = max(X.max(), Y.max()) - min(X.min(), Y.min())
    if L == 0.0:
        return np.ones((ny, nx))
    C1 = (0.01 * L) ** 2
    C2 = (0.03 * L) ** 2
    out = np.empty((ny, nx))
    for ty in range(ny):
        for tx in range(nx):
            x = X[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile]
            y = Y[ty * tile:(ty + 1) * tile, tx * tile:(tx + 1) * tile]
            mx, my = x.mean(), y.mean()
            vx = ((x - mx) ** 2).mean()
            vy = ((y - my) ** 2).mean()
            cxy = ((x - mx) * (y - my)).mean()
            S = ((2 * mx * my + C1) * (2 * cxy + C2)) / ((mx * mx + my * my + C1) * (vx + vy + C2))
            out[ty, tx] = min(1.0, max(0.0, 0.5 * (1.0 + S)))
    return out


def periodic_score(series):
    """max over fundamental f and harmonic count h of (sum_{j<=h, jf<=n/2} P_{jf}) / sqrt(h),
    P the DFT power of the mean-removed series of length n."""
    x = np.asarray(series, dtype=np.float64)
    n = x.size
    d = x - x.mean()
    tau = np.arange(n)
    P = np.zeros(n // 2 + 1)
    for f in range(1, n // 2 + 1):
        P[f] = abs(np.sum(d * np.exp(-2j * math.pi * f * tau / n))) ** 2
    best = -np.inf
    for f in range(1, n // 2 + 1):
        for h in HARMONICS:
            s = sum(P[j * f] for j in range(1, h + 1) if j * f <= n // 2)
            best = max(best, s / math.sqrt(h))
    return best


def zscore(a):
    a = np.asarray(a, dtype=np.float64)
    sd = a.std()
    return np.zeros_like(a) if sd == 0 else (a - a.mean()) / sd


def components8(mask):
    """8-connected components of a boolean tile mask (breadth-first search)."""
    ny, nx = mask.shape
    lab = -np.ones(mask.shape, dtype=np.int64)
    comps = []
    for y in range(ny):
        for x in range(nx):
            if mask[y, x] and lab[y, x] < 0:
                lab[y, x] = len(comps)
                todo = [(y, x)]
                cells = []
                while todo:
                    cy, cx = todo.pop()
                    cells.append((cy, cx))
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            yy, xx = cy + dy, cx + dx
                            if 0 <= yy < ny and 0 <= xx < nx and mask[yy, xx] and lab[yy, xx] < 0:
                                lab[yy, xx] = len(comps)
                                todo.append((yy, xx))
                comps.append(cells)
    return comps


def window_scores(window):
    """(periodic z, non-periodic z) maps of an (L, ty, tx) window or cube of tLISI maps."""
    w = np.asarray(window, dtype=np.float64)
    ny, nx = w.shape[1:]
    per = np.empty((ny, nx))
    for y in range(ny):
        for x in range(nx):
            per[y, x] = periodic_score(w[:, y, x])
    nonper = (1.0 - w).sum(axis=0)
    return zscore(per), zscore(nonper)


def detect(window, t, tile=32, z_periodic=5.0, z_nonperiodic=4.0):
    """Candidate boxes (t, x0, y0, x1, y1) in pixels of one window (or the whole
    cube) of tLISI maps ending at snapshot t."""
    zp, zn = window_scores(window)
    mask = (zp > z_periodic) | (zn > z_nonperiodic)
    boxes = []
    for cells in components8(mask):
        ys = [c[0] for c in cells]; xs = [c[1] for c in cells]
        boxes.append((t, tile * min(xs), tile * min(ys), tile * max(xs) + tile - 1,
                      tile * max(ys) + tile - 1))
    boxes.sort(key=lambda b: (b[0], b[2], b[1], b[4], b[3]))
    return boxes, zp, zn
