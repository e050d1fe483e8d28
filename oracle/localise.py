"""Full-resolution localisation of a candidate (FP64 oracle; test
infrastructure only: the product path never imports it).

Section 2 and Section 6: within each candidate box, a difference image of two
time-adjacent snapshots is searched: the local median background is
subtracted, source pixels are selected with a local 5 sigma threshold, the
connected component holding the brightest pixel is required to look like a
Gaussian source, and its intensity-weighted centroid is turned into RA/Dec
through the image's SIN projection.  The paper names the steps but not their
details; the readings here (each a documented choice):

- D = I_b - I_a in FP32 (the images' type), the box inclusive of its corners;
- background: the lower median of the box's n values, element (n - 1) // 2 of
  the sorted values; sigma = 1.4826 MAD, MAD the lower median of |D - med|
  (both are elements of FP32 arrays, so the selections are exact);
- the brightest pixel p*: largest |D - med|, the first in row-major order on
  ties; s = +1 if D - med >= 0 at p* else -1 (a pulsar may switch off);
- source pixels: s (D - med) > 5 sigma (FP64); the component: 8-connected
  source pixels reached from p* (none if p* itself is not a source pixel);
- Gaussian-like (optional): at least 3 pixels, the intensity-weighted second
  moments (weights w = s (D - med)) have a smaller eigenvalue > 0 and an axis
  ratio sqrt(l1 / l2) <= 3, and p* lies within 1.5 pixels of the centroid;
- centroid (xc, yc) = sum w (j1, j2) / sum w in image pixels (0-based j1
  across, j2 up); direction cosines l = -D (xc - N/2), m = D (yc - N/2)
  (D = cell in radians, the imager's pixel convention); inverse SIN:
  n = sqrt(1 - l^2 - m^2), dec = asin(m cos dec0 + n sin dec0),
  ra = ra0 + atan2(l, n cos dec0 - m sin dec0).
- The adjacent pair: the tLISI map with the smallest mean over the box's
  tiles marks the strongest change; map k compares (I_{k+1} - I_k) with
  (I_{k+2} - I_{k+1}) and the newer difference, (k + 1, k + 2), is searched.
"""
from __future__ import annotations

import math

import numpy as np

MAD_TO_SIGMA = 1.4826
N_SIGMA = 5.0
MAX_AXIS_RATIO = 3.0
MAX_PEAK_OFFSET = 1.5


def strongest_map(cube, box, tile=32):
    """Index k of the tLISI map (cube[k], oldest first) with the smallest mean over
    the tiles of box (t, x0, y0, x1, y1); the first such k on ties."""
    _, x0, y0, x1, y1 = box
    c = np.asarray(cube, dtype=np.float64)[:, y0 // tile:y1 // tile + 1, x0 // tile:x1 // tile + 1]
    m = c.reshape(c.shape[0], -1).sum(axis=1)
    return int(np.argmin(m))


def lower_median(v):
    s = np.sort(np.asarray(v).ravel())
    return s[(s.size - 1) // 2]


def components_from(mask, start):
    """The 8-connected set of True cells of mask reached from start (row, col)."""
    ny, nx = mask.shape
    seen = np.zeros(mask.shape, dtype=bool)
    if not mask[start]:
        return seen
    todo = [start]
    seen[start] = True
    while todo:
        y, x = todo.pop()
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yy, xx = y + dy, x + dx
                if 0 <= yy < ny and 0 <= xx < nx and mask[yy, xx] and not seen[yy, xx]:
                    seen[yy, xx] = True
                    todo.append((yy, xx))
    return seen


def pixel_to_radec(xc, yc, n_pix, cell_deg, ra0_deg, dec0_deg):
    d = math.radians(cell_deg)
    l = -d * (xc - n_pix / 2)
    m = d * (yc - n_pix / 2)
    n = math.sqrt(max(0.0, 1.0 - l * l - m * m))
    dec0 = math.radians(dec0_deg)
    dec = math.asin(m * math.cos(dec0) + n * math.sin(dec0))
    ra = math.radians(ra0_deg) + math.atan2(l, n * math.cos(dec0) - m * math.sin(dec0))
    return math.degrees(ra) % 360.0, math.degrees(dec)


def localise(img_a, img_b, box, n_pix, cell_deg, ra0_deg, dec0_deg, morph=True):
    """Position of the source in box (t, x0, y0, x1, y1) of the difference img_b - img_a."""
    _, x0, y0, x1, y1 = box
    a = np.asarray(img_a, dtype=np.float32)[y0:y1 + 1, x0:x1 + 1]
    b = np.asarray(img_b, dtype=np.float32)[y0:y1 + 1, x0:x1 + 1]
    D = b - a                                             # FP32
    med = lower_median(D)
    r = D - med                                           # FP32
    mad = lower_median(np.abs(r))
    sigma = MAD_TO_SIGMA * float(mad)
    flat = np.abs(r).ravel()
    k = int(np.argmax(flat))                              # first maximum in row-major order
    py, px = divmod(k, D.shape[1])
    s = 1.0 if r[py, px] >= 0 else -1.0
    w = s * r.astype(np.float64)
    sel = w > N_SIGMA * sigma
    comp = components_from(sel, (py, px))
    out = dict(valid=False, xc=math.nan, yc=math.nan, ra=math.nan, dec=math.nan, peak=float(w[py, px]),
               sigma=sigma, n_pix=int(comp.sum()), peak_x=x0 + px, peak_y=y0 + py, morph_ok=False)
    if not comp.any():
        return out
    ys, xs = np.nonzero(comp)
    ww = w[ys, xs]
    W = ww.sum()
    xc = (ww * (x0 + xs)).sum() / W
    yc = (ww * (y0 + ys)).sum() / W
    cxx = (ww * (x0 + xs - xc) ** 2).sum() / W
    cyy = (ww * (y0 + ys - yc) ** 2).sum() / W
    cxy = (ww * (x0 + xs - xc) * (y0 + ys - yc)).sum() / W
    tr, det = cxx + cyy, cxx * cyy - cxy * cxy
    disc = math.sqrt(max(0.0, tr * tr / 4 - det))
    l1, l2 = tr / 2 + disc, tr / 2 - disc
    morph_ok = (comp.sum() >= 3 and l2 > 0 and math.sqrt(l1 / l2) <= MAX_AXIS_RATIO
                and math.hypot(x0 + px - xc, y0 + py - yc) <= MAX_PEAK_OFFSET)
    ra, dec = pixel_to_radec(xc, yc, n_pix, cell_deg, ra0_deg, dec0_deg)
    out.update(xc=xc, yc=yc, ra=ra, dec=dec, morph_ok=bool(morph_ok), valid=bool(morph_ok or not morph))
    return out
