"""Pins of the oracle's re-projection (§3.3, App. A, eq. 9)."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import toi


def _basis(sigma_h=40.0, seed=0):
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=8, n_chan=6, n_pix=32, sigma_h_m=sigma_h, seed=seed)
    return toi.snapshot_basis(toi.select_samples(S.make_snapshot(wl, 0)).b)


def test_untilted_basis_is_the_identity_map():
    rng = np.random.default_rng(0)
    N = 40
    img = rng.normal(size=(N, N))
    out, valid = toi.reproject(img, np.eye(3), N, 0.01)
    assert valid[:N - 1, :N - 1].all()
    np.testing.assert_allclose(out[valid], img[valid], atol=1e-12)


def test_reduced_mapping_equals_wcs_sin_chain():
    rng = np.random.default_rng(1)
    N, cell = 4096, 0.000732
    for xi, eta in ((0.0, 0.0), (-0.2264, -0.0285), (0.7, -0.4), (1e-3, 2e-3)):
        p1 = rng.integers(1, N + 1, 300).astype(float)
        p2 = rng.integers(1, N + 1, 300).astype(float)
        p1[0], p2[0] = N / 2 + 1, N / 2 + 1                   # the projection centre (h = 0)
        p1[1], p2[1] = N / 2 + 1, 7                           # x = 0, y < 0
        a1, a2 = toi.reduced_sin_map(p1, p2, xi, eta, N, cell)
        b1, b2 = toi.wcs_sin_chain(p1, p2, xi, eta, N, cell)
        assert np.abs(a1 - b1).max() < 1e-8 and np.abs(a2 - b2).max() < 1e-8


def test_literal_yhat_sign_would_mirror_an_untilted_plane():
    # With xi = eta = 0 the reduced map must be the identity.  The printed
    # yhat = -y/h would give y' = -y, i.e. p2' = N + 2 - p2 (a mirror); the
    # App. A chain fixes the sign used by the oracle.
    N, cell = 64, 0.01
    p1 = np.arange(1, N + 1, dtype=float); p2 = np.arange(1, N + 1, dtype=float)[::-1]
    a1, a2 = toi.reduced_sin_map(p1, p2, 0.0, 0.0, N, cell)
    np.testing.assert_allclose(a1, p1, atol=1e-12)
    np.testing.assert_allclose(a2, p2, atol=1e-12)


def test_exact_mapping_is_reduced_map_then_in_plane_block():
    bas = _basis()
    V = bas.V
    N, cell = 256, 0.005
    d = math.radians(cell)
    rng = np.random.default_rng(2)
    j1 = rng.integers(0, N, 200); j2 = rng.integers(0, N, 200)
    u1, u2, ok = toi.reproject_coords(V, N, cell, j1, j2)
    a1, a2 = toi.reduced_sin_map(j1 + 1.0, j2 + 1.0, bas.xi, bas.eta, N, cell)
    # slant coordinates (radians) of the reduced map, then the 2 x 2 block of V
    a = -d * (a1 - (N / 2 + 1)); b = d * (a2 - (N / 2 + 1))
    t1 = V[0, 0] * a + V[0, 1] * b
    t2 = V[1, 0] * a + V[1, 1] * b
    np.testing.assert_allclose(u1, N / 2 - t1 / d, atol=1e-9)
    np.testing.assert_allclose(u2, N / 2 + t2 / d, atol=1e-9)


def test_reprojected_exact_image_equals_standard_grid_dft():
    # b . s = r . t (eq. 10-1): evaluating eq. (10) at t = V s reproduces the
    # standard-grid sum over b for every output pixel, whatever the basis.
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=10, n_chan=8, n_pix=24, sigma_h_m=50.0, cell_arcsec=120.0)
    snap = S.make_snapshot(wl, 0)
    smp = toi.select_samples(snap)
    l1, m1 = toi.pixel_offsets(wl.n_pix, wl.cell_deg)
    l, m = np.meshgrid(l1, m1)
    nm1 = np.sqrt(1 - l * l - m * m) - 1
    std = np.real(smp.x @ np.exp(2j * math.pi * (np.outer(smp.b[:, 0], l.ravel())
                                                  + np.outer(smp.b[:, 1], m.ravel())
                                                  + np.outer(smp.b[:, 2], nm1.ravel()))))
    for seed_rot in (None, 0.7, -2.0):
        bas = toi.snapshot_basis(smp.b)
        V = bas.V.copy()
        if seed_rot is not None:                       # any in-plane rotation of e1, e2
            c, s_ = math.cos(seed_rot), math.sin(seed_rot)
            V[:2] = np.array([[c, s_], [-s_, c]]) @ V[:2]
        om = toi.basis_from_V(V).omega
        r = toi.rotate(V, smp.b)
        t = V @ np.stack([l.ravel(), m.ravel(), nm1.ravel()])
        t3 = toi.t3_of(t[0], t[1], V)
        val = toi.tplane_at(r, smp.x, smp.W, om, t[0], t[1], t3)
        np.testing.assert_allclose(val * om * smp.W, std, atol=1e-9 * np.abs(smp.x).sum())


def test_reprojection_of_gridded_tplane_approaches_standard_dft():
    # informational bound: bilinear interpolation of a well-sampled t-plane image
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=10, n_chan=8, n_pix=48, sigma_h_m=20.0, cell_arcsec=20.0)
    res = toi.image_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, exact=True)
    smp = res.samples
    l1, m1 = toi.pixel_offsets(wl.n_pix, wl.cell_deg)
    l, m = np.meshgrid(l1, m1)
    nm1 = np.sqrt(1 - l * l - m * m) - 1
    std = np.real(smp.x @ np.exp(2j * math.pi * (np.outer(smp.b[:, 0], l.ravel())
                                                  + np.outer(smp.b[:, 1], m.ravel())
                                                  + np.outer(smp.b[:, 2], nm1.ravel()))))
    std = std.reshape(l.shape) / (res.basis.omega * smp.W)
    v = res.valid
    assert v.mean() > 0.8
    assert np.abs(res.image[v] - std[v]).max() < 0.15 * np.abs(std).max()


def _bilinear_form(a, b, c, d, n):
    """img[j2][j1] = a + b j1 + c j2 + d j1 j2 (reproduced exactly by bilinear interpolation)."""
    j1 = np.arange(n, dtype=np.float64)[None, :]
    j2 = np.arange(n, dtype=np.float64)[:, None]
    return a + b * j1 + c * j2 + d * j1 * j2


def test_bilinear_reproduces_a_bilinear_form_at_fractional_positions():
    # distinct coefficients on j1 and j2: a swap of the fractions, of the axes
    # or of two corner weights changes the value
    N = 37
    a, b, c, d = 0.3, 1.7, -2.9, 0.011
    img = _bilinear_form(a, b, c, d, N)
    rng = np.random.default_rng(11)
    u1 = rng.uniform(0.0, N - 1.0, 500)
    u2 = rng.uniform(0.0, N - 1.0, 500)
    u1[:3] = [0.0, 35.999999, 12.5]
    u2[:3] = [35.25, 0.0, 7.0]                             # integer and edge positions
    v, valid = toi.bilinear(img, u1, u2)
    assert valid.all()
    np.testing.assert_allclose(v, a + b * u1 + c * u2 + d * u1 * u2, atol=1e-11)
    # outside: any neighbour beyond the image -> 0 and invalid
    v2, valid2 = toi.bilinear(img, np.array([-0.01, N - 1.0, 3.0, 3.0]), np.array([3.0, 3.0, -1e-9, N - 0.5]))
    assert not valid2.any() and (v2 == 0).all()


def test_reprojection_of_a_bilinear_tplane_is_exact_at_the_mapped_positions():
    # With a tilted basis the output pixel (j1, j2) reads the transformed plane
    # at (u1, u2) = reproject_coords; for a bilinear-form t-plane the
    # re-projected value is the form at exactly that position.
    bas = _basis(sigma_h=60.0, seed=3)
    assert abs(bas.xi) + abs(bas.eta) > 1e-3
    N, cell = 64, 0.05
    a, b, c, d = -1.25, 0.75, 2.5, -0.004
    tp = _bilinear_form(a, b, c, d, N)
    img, valid = toi.reproject(tp, bas.V, N, cell)
    u1, u2, ok = toi.reproject_coords(bas.V, N, cell)
    assert valid.mean() > 0.5
    want = a + b * u1 + c * u2 + d * u1 * u2
    np.testing.assert_allclose(img[valid], want[valid], atol=1e-10)
    assert (img[~valid] == 0).all()
