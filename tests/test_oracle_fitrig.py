"""Pins of the oracle's tLISI stand-in and window detection (FITrig stage)."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import fitrig


def _imgs(seed, n=64):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=(n, n)) for _ in range(3)]


def test_identical_differences_give_one():
    a, b, _ = _imgs(0)
    c = b + (b - a)                       # X == Y exactly
    np.testing.assert_allclose(fitrig.tlisi(a, b, c, tile=16), 1.0, atol=1e-12)
    # constant images: L = 0, identical by definition
    z = np.zeros((64, 64))
    np.testing.assert_array_equal(fitrig.tlisi(z, z, z, tile=16), 1.0)


def test_range_symmetry_and_anticorrelation():
    a, b, c = _imgs(1)
    t = fitrig.tlisi(a, b, c, tile=16)
    assert t.shape == (4, 4) and np.all((t >= 0) & (t <= 1))
    # swapping the two difference images leaves the index unchanged
    X, Y = b - a, c - b
    t2 = fitrig.tlisi(np.zeros_like(X), Y, X + Y, tile=16)
    np.testing.assert_allclose(t, t2, atol=1e-12)
    # Y = -X with zero-mean tiles: strongly dissimilar
    X = X - X.reshape(4, 16, 4, 16).mean(axis=(1, 3)).repeat(16, 0).repeat(16, 1)
    ta = fitrig.tlisi(np.zeros_like(X), X, np.zeros_like(X), tile=16)
    assert np.all(ta < 0.5)


def test_tile_statistics_by_explicit_sums():
    a, b, c = _imgs(2, n=32)
    tile = 8
    X, Y = b - a, c - b
    L = max(X.max(), Y.max()) - min(X.min(), Y.min())
    C1, C2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    t = fitrig.tlisi(a, b, c, tile=tile)
    for ty in range(4):
        for tx in range(4):
            sx = sy = sxx = syy = sxy = 0.0
            for y in range(ty * tile, (ty + 1) * tile):
                for x in range(tx * tile, (tx + 1) * tile):
                    sx += X[y, x]; sy += Y[y, x]
                    sxx += X[y, x] ** 2; syy += Y[y, x] ** 2; sxy += X[y, x] * Y[y, x]
            n = tile * tile
            mx, my = sx / n, sy / n
            vx, vy, cxy = sxx / n - mx * mx, syy / n - my * my, sxy / n - mx * my
            S = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
            assert t[ty, tx] == pytest.approx(0.5 * (1 + S), abs=1e-12)


def test_transient_tile_has_lowest_index():
    rng = np.random.default_rng(3)
    base = rng.normal(scale=0.01, size=(64, 64))
    imgs = [base + rng.normal(scale=0.01, size=base.shape) for _ in range(3)]
    imgs[2][40:44, 20:24] += 1.0          # appears only in the newest image
    t = fitrig.tlisi(*imgs, tile=16)
    assert np.unravel_index(np.argmin(t), t.shape) == (2, 1)


def test_periodic_score_closed_form():
    A = 0.3
    tau = np.arange(16)
    x = 0.8 + A * np.cos(2 * math.pi * 4 * tau / 16)
    # P_4 = (A * 16 / 2)^2, every other bin 0; best is h = 1 at f = 4
    assert fitrig.periodic_score(x) == pytest.approx((A * 8) ** 2, rel=1e-12)
    y = 0.8 + A * (np.cos(2 * math.pi * 2 * tau / 16) + np.cos(2 * math.pi * 4 * tau / 16))
    # f = 2 with h = 2 collects P_2 + P_4 = 2 (8A)^2, normalised by sqrt 2
    assert fitrig.periodic_score(y) == pytest.approx(2 * (A * 8) ** 2 / math.sqrt(2), rel=1e-12)


def test_periodic_score_closed_form_whole_run_length():
    # the whole-cube statistic: a series of any length L (here 150, not a power
    # of two); a cosine of integer frequency f0 has P_f0 = (A L / 2)^2 and no
    # other power, so the best score is h = 1 at f0 unless f0's harmonics add
    A, L = 0.2, 150
    tau = np.arange(L)
    x = 0.9 + A * np.cos(2 * math.pi * 7 * tau / L + 0.4)
    assert fitrig.periodic_score(x) == pytest.approx((A * L / 2) ** 2, rel=1e-10)
    # fundamental 5 with harmonics 10, 15, 20: h = 4 collects 4 (A L / 2)^2 / 2
    y = 0.9 + A * sum(np.cos(2 * math.pi * 5 * j * tau / L) for j in (1, 2, 3, 4))
    assert fitrig.periodic_score(y) == pytest.approx(4 * (A * L / 2) ** 2 / 2, rel=1e-10)
    # brute-force DFT power of a random series equals numpy's FFT
    r = np.random.default_rng(8).random(L)
    d = r - r.mean()
    P = np.abs(np.fft.rfft(d)) ** 2
    best = max(sum(P[j * f] for j in range(1, h + 1) if j * f <= L // 2) / math.sqrt(h)
               for f in range(1, L // 2 + 1) for h in (1, 2, 4, 8))
    assert fitrig.periodic_score(r) == pytest.approx(best, rel=1e-9)


def test_components_match_scipy_label():
    rng = np.random.default_rng(4)
    for _ in range(20):
        mask = rng.random((20, 24)) < 0.2
        comps = fitrig.components8(mask)
        lab, n = ndimage.label(mask, structure=np.ones((3, 3)))
        assert len(comps) == n
        got = sorted(sorted(c) for c in comps)
        want = sorted(sorted(zip(*np.nonzero(lab == k))) for k in range(1, n + 1))
        assert got == [[tuple(map(int, p)) for p in w] for w in want]


def test_detect_planted_pulsar_and_ramp():
    rng = np.random.default_rng(5)
    w = 1.0 - np.abs(rng.normal(scale=0.01, size=(16, 16, 16)))
    tau = np.arange(16)
    w[:, 3, 4] = 0.6 + 0.3 * np.cos(2 * math.pi * 4 * tau / 16)       # periodic tile
    w[:, 4, 5] = 0.6 + 0.3 * np.cos(2 * math.pi * 4 * tau / 16)       # diagonal neighbour: same box
    w[:, 12, 10] -= 0.2                                                # steady drop: non-periodic
    boxes, zp, zn = fitrig.detect(w, t=40, tile=32)
    assert boxes == [(40, 128, 96, 32 * 5 + 31, 32 * 4 + 31), (40, 320, 384, 351, 415)]
