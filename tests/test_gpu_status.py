"""The device status word (toi_plan_info) for every data-dependent condition,
each forced from the host: the image and transformed plane are all zero, the
bit is set, and the next snapshot on the same context images normally."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import toi as O

from gpu_helpers import IMAGE_TOL, max_rel_err

pytestmark = pytest.mark.gpu


def _wl(**kw):
    base = dict(n_ant=10, n_chan=24, n_pix=64, cell_arcsec=60.0, sigma_h_m=20.0, n_steady=3)
    base.update(kw)
    return S.scaled(S.WORKLOADS["tiny"], **base)


def _image(im, snap):
    from paper_2512_06254_amd import toi as T
    im.grid(T.to_device(snap))
    img, tp = im.image(tplane=True)
    return img.cpu().numpy(), tp.cpu().numpy(), im.plan_info()


def _recovers(im, wl, **plan):
    """A normal snapshot on the same context afterwards images like the oracle."""
    snap = S.make_snapshot(wl, 0)
    img, tp, info = _image(im, snap)
    res = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, **plan)
    assert info["status"] == 0
    assert max_rel_err(tp, res.tplane) <= IMAGE_TOL


def test_degenerate_basis_edge_on_plane():
    from paper_2512_06254_amd import toi as T
    wl = _wl()
    snap = S.make_snapshot(wl, 0)
    snap["uvw"] = snap["uvw"].copy()
    snap["uvw"][:, 0] = 0.0          # every baseline in the v-w plane: the normal is the u axis, V33 = 0
    bas = O.snapshot_basis(O.select_samples(snap).b)
    assert abs(bas.V[2, 2]) < 1e-6
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=4)
    img, tp, info = _image(im, snap)
    print(f"[degenerate] status {info['status']} V33 {info['V'][2, 2]:.2e}", flush=True)
    assert info["status"] & T.STATUS_DEGENERATE
    assert not img.any() and not tp.any()
    _recovers(im, wl, n_slab=1, K=4)
    im.close()


def test_planes_beyond_capacity():
    from paper_2512_06254_amd import toi as T
    wl = _wl()
    snap = S.make_snapshot(wl, 0)
    res = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=2)     # automatic K >= 8
    assert res.plan.planes > 8
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=2, cheb_k=0, max_planes=8)
    img, tp, info = _image(im, snap)
    print(f"[planes] status {info['status']} plan {info['n_slab']} x {info['K']}", flush=True)
    assert info["status"] & T.STATUS_PLANES
    assert info["n_slab"] * info["K"] == res.plan.planes
    assert not img.any() and not tp.any()
    im.close()


def test_bin_list_overflow_gives_zero_image():
    from paper_2512_06254_amd import toi as T
    wl = _wl()
    snap = S.make_snapshot(wl, 0)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=4, bin_cap=16)
    img, tp, info = _image(im, snap)
    print(f"[overflow] status {info['status']}", flush=True)
    assert info["status"] == T.STATUS_OVERFLOW
    assert not img.any() and not tp.any()
    # a snapshot whose lists fit: three rows, one work item each
    small = {k: (v[:3] if k in ("uvw", "vis", "ant1", "ant2") and v is not None else v) for k, v in snap.items()}
    img, tp, info = _image(im, small)
    res = O.image_snapshot(small, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=4)
    assert info["status"] == 0 and max_rel_err(tp, res.tplane) <= IMAGE_TOL
    im.close()
    with pytest.raises(T.ToiError):
        T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, bin_cap=-1)
