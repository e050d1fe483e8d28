"""Pins of the oracle's dirty images (§3.2, §3.4, App. B) against closed forms,
brute force, the paper's Table "cheby" and the truncation bound."""
import math
import os

import numpy as np
import pytest

import synth_inputs as S
from oracle import gridded, toi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _wl(**kw):
    base = dict(n_ant=8, n_chan=6, n_pix=32, n_steady=2, cell_arcsec=60.0, sigma_h_m=20.0)
    base.update(kw)
    return S.scaled(S.WORKLOADS["tiny"], **base)


def _flat_snapshot(wl, flux=1.75):
    """A point source at the phase centre: every visibility equals its flux."""
    snap = S.make_snapshot(wl, 0, with_noise=False)
    snap["vis"] = np.full(snap["vis"].shape, flux, dtype=np.complex64)
    if wl.n_corr == 4:
        snap["vis"][:, :, 1:3] = 0
    return snap


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n_corr", [1, 4])
def test_point_source_at_phase_centre_gives_flux_over_omega(n_corr):
    wl = _wl(n_corr=n_corr)
    snap = _flat_snapshot(wl)
    c = wl.n_pix // 2
    for mode, exact in ((2, False), (3, False), (3, True)):
        res = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=mode, exact=exact, n_slab=1, K=8)
        want = 1.75 / res.basis.omega
        assert res.tplane[c, c] == pytest.approx(want, rel=1e-12)
        assert res.image[c, c] == pytest.approx(want, rel=1e-12)
        assert np.argmax(res.image) == c * wl.n_pix + c


def test_offset_source_peaks_at_its_pixel():
    wl = _wl(n_ant=16, n_chan=16, n_pix=48, sigma_h_m=30.0)
    snap = S.make_snapshot(wl, 0, with_noise=False)
    d = math.radians(wl.cell_deg)
    j1, j2 = 31, 17
    l0, m0 = -d * (j1 - wl.n_pix / 2), d * (j2 - wl.n_pix / 2)
    snap["vis"] = S.predict(snap["uvw"], snap["freq"], [l0], [m0], [2.5], 1).numpy()
    res = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, exact=True)
    assert np.unravel_index(np.argmax(res.image), res.image.shape) == (j2, j1)
    # eq. (10) at the source's transformed coordinates t = V s is exactly S / omega
    n0 = math.sqrt(1 - l0 * l0 - m0 * m0)
    t = res.basis.V @ np.array([l0, m0, n0 - 1])
    t3 = toi.t3_of(t[0], t[1], res.basis.V)
    val = toi.tplane_at(res.r, res.samples.x, res.samples.W, res.basis.omega, t[0], t[1], t3)
    assert val[0] == pytest.approx(2.5 / res.basis.omega, rel=1e-10)


def test_t3_branch_lies_on_the_sphere_and_matches_Vs():
    wl = _wl(sigma_h_m=40.0)
    V = toi.snapshot_basis(toi.select_samples(S.make_snapshot(wl, 0)).b).V
    rng = np.random.default_rng(3)
    for Vc in (V, V * np.array([[1], [-1], [-1]])):      # both signs of V33, still a rotation
        assert abs(toi.t3_of(0.0, 0.0, Vc)) < 1e-15
        l, m = rng.uniform(-0.05, 0.05, (2, 200))
        s = np.stack([l, m, np.sqrt(1 - l * l - m * m) - 1])
        t = Vc @ s
        t3 = toi.t3_of(t[0], t[1], Vc)
        np.testing.assert_allclose(t3, t[2], atol=1e-15)
        np.testing.assert_allclose((t[0] + Vc[0, 2]) ** 2 + (t[1] + Vc[1, 2]) ** 2
                                   + (t3 + Vc[2, 2]) ** 2, 1.0, atol=1e-14)


def test_coplanar_snapshot_makes_3d_equal_2d():
    wl = _wl(sigma_h_m=0.0)
    snap = S.make_snapshot(wl, 0)
    i2 = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=2).tplane
    i3 = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3).tplane
    i3x = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, exact=True).tplane
    peak = np.abs(i2).max()
    assert np.abs(i3 - i2).max() < 1e-10 * peak
    assert np.abs(i3x - i2).max() < 1e-10 * peak


def test_brute_force_dft_on_tiny_input():
    wl = _wl(n_ant=4, n_chan=3, n_pix=8, sigma_h_m=40.0)
    snap = S.make_snapshot(wl, 0)
    res = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=2, K=3)
    r, x, W, om, V = res.r, res.samples.x, res.samples.W, res.basis.omega, res.basis.V
    d = math.radians(wl.cell_deg)
    N = wl.n_pix
    i2 = np.zeros((N, N)); i3 = np.zeros((N, N))
    plan = res.plan
    for j2 in range(N):
        for j1 in range(N):
            t1, t2 = -d * (j1 - N / 2), d * (j2 - N / 2)
            t3 = -V[2, 2] + math.sqrt(1 - (t1 + V[0, 2]) ** 2 - (t2 + V[1, 2]) ** 2)
            s2 = 0j; s3 = 0j
            for q in range(x.size):
                s2 += x[q] * np.exp(2j * math.pi * (r[q, 0] * t1 + r[q, 1] * t2))
                s3 += x[q] * np.exp(2j * math.pi * (r[q, 0] * t1 + r[q, 1] * t2 + r[q, 2] * t3))
            i2[j2, j1] = s2.real / (om * W)
            i3[j2, j1] = s3.real / (om * W)
    np.testing.assert_allclose(toi.image_2d(r, x, W, om, N, wl.cell_deg), i2, atol=1e-12)
    np.testing.assert_allclose(toi.image_3d_exact(r, x, W, om, V, N, wl.cell_deg), i3, atol=1e-12)
    # Chebyshev moments: brute-force slab sums with T_k(s) = cos(k arccos s)
    M = toi.moments(r, x, plan, N, wl.cell_deg)
    j1, j2 = 5, 2
    t1, t2 = -d * (j1 - N / 2), d * (j2 - N / 2)
    for p in range(plan.n_slab):
        for k in range(plan.K):
            acc = 0j
            for q in range(x.size):
                pq = min(plan.n_slab - 1, int((r[q, 2] - plan.r3min) // (2 * plan.dr3)))
                if pq != p:
                    continue
                sq = (r[q, 2] - (plan.r3min + (2 * p + 1) * plan.dr3)) / plan.dr3
                acc += math.cos(k * math.acos(max(-1, min(1, sq)))) * x[q] * np.exp(
                    2j * math.pi * (r[q, 0] * t1 + r[q, 1] * t2))
            assert abs(M[p, k, j2, j1] - acc) < 1e-12 * max(1.0, abs(acc))


def test_truncation_bound_and_convergence():
    wl = _wl(n_pix=24, sigma_h_m=30.0, cell_arcsec=120.0)
    snap = S.make_snapshot(wl, 0)
    ex = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, exact=True)
    s, b = ex.samples, ex.basis
    assert 0.5 < ex.plan.alpha_slab < 5
    for K in (2, 3, 4, 6, 8, 12, 16):
        plan = toi.make_plan(ex.r[:, 2], b.V, wl.n_pix, wl.cell_deg, n_slab=1, K=K)
        ik = toi.image_3d_cheb(ex.r, s.x, s.W, b.omega, b.V, plan, wl.n_pix, wl.cell_deg)
        err = np.abs(ik - ex.tplane).max()
        eps = toi.cheb_sampled_error(plan.alpha_slab, K, n_grid=2049)
        assert err <= np.abs(s.x).sum() / (b.omega * s.W) * eps * 1.001 + 1e-13
    assert err < 1e-10 * np.abs(ex.tplane).max()


# ---------------------------------------------------------------- Chebyshev rule

def _golden_cheby():
    rows = []
    with open(os.path.join(GOLDEN, "cheby_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, phi, ns, a, k, nk = line.split()
                rows.append((name, float(phi), int(ns), float(a), int(k), int(nk)))
    return rows


@pytest.mark.parametrize("row", _golden_cheby(), ids=lambda r: r[0])
def test_parameter_rule_reproduces_table_cheby(row):
    _, phi, ns, a, k, nk = row
    # choose scales with 2 pi t3max (r3max - r3min) / 2 = Phi_max
    plan = toi.plan_from_scales(t3max=phi / (2 * math.pi), r3min=-0.5, r3max=1.5)
    assert plan.phimax == pytest.approx(phi, rel=1e-12)
    assert plan.n_slab == ns
    assert round(plan.alpha_slab, 2) == a
    assert plan.K == k
    assert plan.planes == nk


def test_jacobi_anger_coefficients():
    s = np.linspace(-1, 1, 41)
    for alpha in (0.0, 0.5, 5.0, 10.0, -3.0):
        # independent coefficients by quadrature of e^{i alpha cos(th)} cos(k th) (App. B2)
        th = (np.arange(4000) + 0.5) * math.pi / 4000
        for k in range(6):
            q = (2 / math.pi) * np.sum(np.exp(1j * alpha * np.cos(th)) * np.cos(k * th)) * (math.pi / 4000)
            if k == 0:
                q *= 0.5
            assert abs(toi.cheb_coeffs(alpha, 6)[k] - q) < 1e-10
        approx = toi.cheb_T(32, s) @ toi.cheb_coeffs(alpha, 32)
        assert np.abs(approx - np.exp(1j * alpha * s)).max() < 1e-13


def test_t3max_and_slab_assignment():
    wl = _wl(sigma_h_m=50.0)
    res = toi.image_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, n_slab=3, K=4)
    plan, r3 = res.plan, res.r[:, 2]
    t1, t2 = toi.pixel_offsets(wl.n_pix, wl.cell_deg)
    brute = max(abs(toi.t3_of(a, b_, res.basis.V)) for a in t1 for b_ in t2)
    assert plan.t3max == brute
    p, s = toi.slab_of(r3, plan)
    assert p.min() == 0 and p.max() == 2
    assert np.all(np.abs(s) <= 1 + 1e-12)
    assert p[np.argmax(r3)] == 2 and p[np.argmin(r3)] == 0


# ---------------------------------------------------------------- gridded variant

def test_es_gridding_matches_direct_moments():
    wl = _wl(n_pix=32, n_chan=8, sigma_h_m=60.0, cell_arcsec=60.0)
    res = toi.image_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, n_slab=2, K=3)
    direct = toi.moments(res.r, res.samples.x, res.plan, wl.n_pix, wl.cell_deg)
    grid = gridded.gridded_moments(res.r, res.samples.x, res.plan, wl.n_pix, wl.cell_deg)
    scale = np.abs(res.samples.x).sum()
    assert np.abs(grid - direct).max() < 1e-6 * scale


def test_subgrid_evaluation_equals_the_full_image_multi_slab():
    """The pixel sub-grid evaluation of the moments and of the Chebyshev/slab
    image (used at full size, where the whole image is out of reach) equals the
    whole-image evaluation at every selected pixel: three slabs, K = 6, columns
    and rows of different counts (a transposed selection would fail)."""
    wl = _wl(n_pix=32, n_ant=10, n_chan=12, sigma_h_m=60.0, cell_arcsec=90.0)
    snap = S.make_snapshot(wl, 0)
    res = toi.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=3, K=6)
    assert res.plan.n_slab == 3 and res.plan.K == 6
    p, _ = toi.slab_of(res.r[:, 2], res.plan)
    assert np.bincount(p, minlength=3).min() > 0            # every slab holds samples
    s, b = res.samples, res.basis
    full_m = toi.moments(res.r, s.x, res.plan, wl.n_pix, wl.cell_deg)
    rng = np.random.default_rng(7)
    j1 = np.sort(rng.choice(wl.n_pix, 9, replace=False))
    j2 = np.sort(rng.choice(wl.n_pix, 5, replace=False))[::-1]
    sub_m = toi.moments(res.r, s.x, res.plan, wl.n_pix, wl.cell_deg, j1=j1, j2=j2)
    np.testing.assert_allclose(sub_m, full_m[:, :, j2][:, :, :, j1], atol=1e-12 * np.abs(full_m).max())
    sub = toi.image_3d_cheb(res.r, s.x, s.W, b.omega, b.V, res.plan, wl.n_pix, wl.cell_deg, j1=j1, j2=j2)
    assert sub.shape == (j2.size, j1.size)
    np.testing.assert_allclose(sub, res.tplane[np.ix_(j2, j1)], atol=1e-12 * np.abs(res.tplane).max())
    # every pixel, one row and one column at a time
    for jj in range(wl.n_pix):
        row = toi.image_3d_cheb(res.r, s.x, s.W, b.omega, b.V, res.plan, wl.n_pix, wl.cell_deg, j2=[jj])
        col = toi.image_3d_cheb(res.r, s.x, s.W, b.omega, b.V, res.plan, wl.n_pix, wl.cell_deg, j1=[jj])
        np.testing.assert_allclose(row[0], res.tplane[jj], atol=1e-12 * np.abs(res.tplane).max())
        np.testing.assert_allclose(col[:, 0], res.tplane[:, jj], atol=1e-12 * np.abs(res.tplane).max())
