"""Pins of the oracle's adjoint and gradients: the dot-product identity and
central finite differences of an image-domain loss."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import adjoint, toi


def _snap(with_gains=True, flags=False, n_corr=4):
    wl = S.scaled(S.WORKLOADS["adjoint"], n_ant=6, n_chan=5, n_pix=16, n_steady=3,
                  cell_arcsec=180.0, n_corr=n_corr, with_gains=with_gains,
                  flag_frac_max=0.3 if flags else 0.0, sigma_h_m=40.0, diameter_m=1000.0)
    return wl, S.make_snapshot(wl, 0)


@pytest.mark.parametrize("mode", [2, 3])
def test_dot_product_identity(mode):
    wl, snap = _snap(flags=True)
    op = adjoint.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=mode, n_slab=2, K=4)
    rng = np.random.default_rng(0)
    n = op.res.samples.n
    for _ in range(3):
        x = rng.normal(size=n) + 1j * rng.normal(size=n)
        y = rng.normal(size=(wl.n_pix, wl.n_pix))
        lhs = np.sum(op.forward(x) * y)
        rhs = np.real(np.sum(np.conj(op.adjoint(y)) * x))
        assert lhs == pytest.approx(rhs, rel=1e-11, abs=1e-12)


def _loss(snap, wl, model, vis=None, gains=None):
    s = dict(snap)
    if vis is not None:
        s["vis"] = vis
    if gains is not None:
        s["gains"] = gains
    # the operator's geometry does not depend on the visibility values
    res = toi.image_snapshot(s, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=4)
    return np.sum((res.image - model) ** 2)


def test_finite_differences_of_vis_and_gains():
    wl, snap = _snap()
    snap["vis"] = snap["vis"].astype(np.complex128)
    snap["gains"] = snap["gains"].astype(np.complex128)
    model = toi.image_snapshot(dict(snap, vis=snap["vis"] * 0.9), wl.n_pix, wl.cell_deg,
                               mode=3, n_slab=1, K=4).image
    op = adjoint.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=4)
    resid = op.forward(op.res.samples.x) - model
    gx = op.adjoint(2.0 * resid)
    gvis, gg = adjoint.vis_gradients(snap, op.res.samples, gx)
    h = 1e-3
    rng = np.random.default_rng(1)
    for _ in range(4):
        r, c, k = rng.integers(0, snap["vis"].shape[0]), rng.integers(0, 5), rng.choice([0, 3])
        for d, part in ((h, np.real), (1j * h, np.imag)):
            vp = snap["vis"].copy(); vp[r, c, k] += d
            vm = snap["vis"].copy(); vm[r, c, k] -= d
            fd = (_loss(snap, wl, model, vis=vp) - _loss(snap, wl, model, vis=vm)) / (2 * h)
            assert fd == pytest.approx(part(gvis[r, c, k]), rel=1e-6, abs=1e-9)
    for a in range(wl.n_ant):
        for d, part in ((h, np.real), (1j * h, np.imag)):
            gp = snap["gains"].copy(); gp[a] += d
            gm = snap["gains"].copy(); gm[a] -= d
            fd = (_loss(snap, wl, model, gains=gp) - _loss(snap, wl, model, gains=gm)) / (2 * h)
            assert fd == pytest.approx(part(gg[a]), rel=1e-4, abs=1e-7)
    # unselected correlations get no gradient
    assert np.all(gvis[:, :, 1:3] == 0)
