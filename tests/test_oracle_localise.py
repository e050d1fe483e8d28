"""Pins of the localisation oracle (oracle/localise.py) against closed forms,
textbook projections and library routines."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import localise as Lz


def _blob(N, x, y, sig_x, sig_y, amp, noise, seed=0):
    rng = np.random.default_rng(seed)
    j2, j1 = np.mgrid[0:N, 0:N]
    g = amp * np.exp(-0.5 * (((j1 - x) / sig_x) ** 2 + ((j2 - y) / sig_y) ** 2))
    return (g + rng.normal(scale=noise, size=(N, N))).astype(np.float32)


def test_centroid_of_a_gaussian_and_the_sign_of_a_dip():
    N = 256
    a = np.zeros((N, N), np.float32)
    b = _blob(N, 100.3, 80.7, 1.5, 1.5, 1.0, 0.005)
    box = (0, 64, 64, 127, 127)
    r = Lz.localise(a, b, box, N, 0.001, 30.0, -40.0)
    assert r["valid"] and r["morph_ok"]
    assert abs(r["xc"] - 100.3) < 0.03 and abs(r["yc"] - 80.7) < 0.03
    assert (r["peak_x"], r["peak_y"]) == (100, 81)
    # the same source switching off: negative difference, same position
    r2 = Lz.localise(b, a, box, N, 0.001, 30.0, -40.0)
    # (the lower median of -D is minus the upper median of D: a slightly different background)
    assert r2["valid"] and r2["xc"] == pytest.approx(r["xc"], abs=1e-4) and r2["peak"] > 0


def test_median_mad_and_component_match_library_routines():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(37, 29)).astype(np.float32)
    assert Lz.lower_median(v) == np.sort(v.ravel())[(v.size - 1) // 2]
    mask = rng.random((40, 30)) < 0.35
    start = tuple(int(i) for i in np.argwhere(mask)[5])
    lab, _ = ndimage.label(mask, structure=np.ones((3, 3)))
    assert np.array_equal(Lz.components_from(mask, start), lab == lab[start])


def test_sin_projection_round_trip_and_phase_centre():
    N, cell, ra0, dec0 = 512, 0.002, 135.0, -40.0
    assert Lz.pixel_to_radec(N / 2, N / 2, N, cell, ra0, dec0) == pytest.approx((ra0, dec0), abs=1e-12)
    for (x, y) in [(10.5, 300.25), (400.0, 20.0), (256.5, 511.0)]:
        ra, dec = Lz.pixel_to_radec(x, y, N, cell, ra0, dec0)
        # forward SIN (textbook): l = cos d sin(a - a0), m = sin d cos d0 - cos d sin d0 cos(a - a0)
        da, d, d0 = math.radians(ra - ra0), math.radians(dec), math.radians(dec0)
        l = math.cos(d) * math.sin(da)
        m = math.sin(d) * math.cos(d0) - math.cos(d) * math.sin(d0) * math.cos(da)
        D = math.radians(cell)
        assert -l / D + N / 2 == pytest.approx(x, abs=1e-9) and m / D + N / 2 == pytest.approx(y, abs=1e-9)


def test_morphology_rejects_a_streak():
    N = 128
    a = np.zeros((N, N), np.float32)
    b = _blob(N, 60.0, 60.0, 5.0, 0.7, 1.0, 0.002, seed=2)
    box = (0, 32, 32, 95, 95)
    r = Lz.localise(a, b, box, N, 0.001, 0.0, 0.0, morph=True)
    assert not r["morph_ok"] and not r["valid"] and r["n_pix"] > 3
    assert Lz.localise(a, b, box, N, 0.001, 0.0, 0.0, morph=False)["valid"]


def test_no_source_pixel_gives_no_position():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(64, 64)).astype(np.float32)
    b = (a + rng.normal(scale=1e-3, size=a.shape)).astype(np.float32)
    r = Lz.localise(a, b, (0, 0, 0, 63, 63), 64, 0.01, 0.0, 0.0)
    assert not r["valid"] and r["n_pix"] == 0


def test_strongest_map_marks_the_change():
    rng = np.random.default_rng(4)
    cube = 1.0 - np.abs(rng.normal(scale=0.01, size=(20, 8, 8)))
    cube[13, 2:4, 5] -= 0.5
    assert Lz.strongest_map(cube, (0, 5 * 32, 2 * 32, 5 * 32 + 31, 3 * 32 + 31)) == 13
