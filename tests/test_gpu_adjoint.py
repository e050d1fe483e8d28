"""GPU adjoint (toi_degrid through the C ABI) against the FP64 oracle adjoint,
the dot-product identity, and the autograd Function."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import adjoint as A
from oracle import toi as O

from gpu_helpers import DENSE, items_per_bin

pytestmark = pytest.mark.gpu


def _setup(n_slab=1, K=8, flags=True, gains=True, n_pix=64, seed=0, dense=False):
    shape = dict(n_ant=8, n_chan=40, n_pix=n_pix, cell_arcsec=60.0, diameter_m=2000.0, sigma_h_m=40.0)
    if dense:
        shape.update(DENSE)
    wl = S.scaled(S.WORKLOADS["adjoint"], n_steady=4, flag_frac_max=0.3 if flags else 0.0, with_gains=gains,
                  seed=seed, **shape)
    snap = S.make_snapshot(wl, 0)
    return wl, snap


def _imager(wl, snap, n_slab, K):
    from paper_2512_06254_amd import toi as T
    n_row, n_chan, n_corr = snap["vis"].shape
    return T.Imager(wl.n_pix, wl.cell_deg, n_row, n_chan, n_corr, n_slab=n_slab, cheb_k=K,
                    n_ant=0 if snap.get("gains") is None else wl.n_ant, max_planes=32)


@pytest.mark.parametrize("n_slab,K,dense", [(1, 8, False), (2, 4, False), (1, 16, False), (1, 16, True)])
def test_adjoint_matches_oracle(n_slab, K, dense):
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup(dense=dense)
    if dense:   # heavy bins: the gather runs over the forward's split work units
        assert items_per_bin(wl).max() > 2 * 64
    op = A.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=n_slab, K=K)
    rng = np.random.default_rng(3)
    y = rng.normal(size=(wl.n_pix, wl.n_pix))
    gx = op.adjoint(y)
    gv_ref, gg_ref = A.vis_gradients(snap, op.res.samples, gx)
    im = _imager(wl, snap, n_slab, K)
    d = T.to_device(snap)
    im.grid(d)
    gv, gg = im.degrid(torch.from_numpy(y.astype(np.float32)).cuda(), d, want_vis=True, want_gains=True)
    gv = gv.cpu().numpy()
    gg = gg.cpu().numpy()
    e_v = np.abs(gv - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(gg - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[adjoint {n_slab}x{K}] grad_vis err {e_v:.3e}  grad_gains err {e_g:.3e}", flush=True)
    assert e_v < 1e-4 and e_g < 1e-4
    im.close()


def test_adjoint_after_a_16x16_bin_forward():
    # forward gridded with 16 x 16 bins (variant 9, 256-cell grid); the gather
    # walks 8 x 8 bins, which toi_degrid builds again from the forward's records
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup(K=16, n_pix=128)
    op = A.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    rng = np.random.default_rng(5)
    y = rng.normal(size=(wl.n_pix, wl.n_pix))
    gx = op.adjoint(y)
    gv_ref, gg_ref = A.vis_gradients(snap, op.res.samples, gx)
    im = _imager(wl, snap, 1, 16)
    im.set_tuning(9)
    d = T.to_device(snap)
    im.grid(d)
    img, tp = im.image(tplane=True)
    ref = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    e_f = np.abs(tp.cpu().numpy() - ref.tplane).max() / np.abs(ref.tplane).max()
    gv, gg = im.degrid(torch.from_numpy(y.astype(np.float32)).cuda(), d, want_vis=True, want_gains=True)
    e_v = np.abs(gv.cpu().numpy() - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(gg.cpu().numpy() - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[adjoint after 16 x 16 bins] forward err {e_f:.3e}  grad_vis err {e_v:.3e}  grad_gains err {e_g:.3e}",
          flush=True)
    assert e_f < 1e-4 and e_v < 1e-4 and e_g < 1e-4
    im.close()


def test_dot_product_identity_through_the_abi():
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup(gains=True)
    im = _imager(wl, snap, 2, 8)
    d = T.to_device(snap)
    rng = np.random.default_rng(4)
    for trial in range(3):
        v = (rng.normal(size=snap["vis"].shape) + 1j * rng.normal(size=snap["vis"].shape)).astype(np.complex64)
        d["vis"] = torch.from_numpy(v).cuda()
        y = torch.from_numpy(rng.normal(size=(wl.n_pix, wl.n_pix)).astype(np.float32)).cuda()
        im.grid(d)
        img = im.image()
        gv, _ = im.degrid(y, d)
        lhs = float((img.double() * y.double()).sum())
        rhs = float((torch.conj(gv.to(torch.complex128)) * d["vis"].to(torch.complex128)).real.sum())
        print(f"[dot] <Gx,y>={lhs:.6e}  Re<x,G^H y>={rhs:.6e}", flush=True)
        assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), 1e-6)
    im.close()


def test_autograd_function_gradients():
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup()
    res = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=8)
    model = torch.from_numpy((0.9 * res.image).astype(np.float32)).cuda()
    im = _imager(wl, snap, 1, 8)
    d = T.to_device(snap)
    vis = d["vis"].clone().requires_grad_(True)
    gains = d["gains"].clone().requires_grad_(True)
    img = T.toi_image(im, d, vis=vis, gains=gains)
    loss = ((img - model) ** 2).sum()
    loss.backward()
    # oracle: same loss, adjoint of 2 (I - model)
    op = A.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=8)
    gx = op.adjoint(2.0 * (res.image - model.cpu().numpy().astype(np.float64)))
    gv_ref, gg_ref = A.vis_gradients(snap, op.res.samples, gx)
    e_v = np.abs(vis.grad.cpu().numpy() - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(gains.grad.cpu().numpy() - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[autograd] grad_vis err {e_v:.3e}  grad_gains err {e_g:.3e}", flush=True)
    assert e_v < 1e-3 and e_g < 1e-3
    im.close()


@pytest.mark.parametrize("n_pix", [32, 128])
def test_adjoint_sizes_whose_first_radix_is_the_pass_radix(n_pix):
    """Grids of 64 and 256 (radix 8 and 16, first stage of full radix): the
    adjoint passes take their input straight in the stage-1 pattern."""
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup(n_pix=n_pix)
    op = A.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=8)
    rng = np.random.default_rng(5)
    y = rng.normal(size=(wl.n_pix, wl.n_pix))
    gx = op.adjoint(y)
    gv_ref, gg_ref = A.vis_gradients(snap, op.res.samples, gx)
    im = _imager(wl, snap, 1, 8)
    d = T.to_device(snap)
    im.grid(d)
    gv, gg = im.degrid(torch.from_numpy(y.astype(np.float32)).cuda(), d, want_vis=True, want_gains=True)
    e_v = np.abs(gv.cpu().numpy() - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(gg.cpu().numpy() - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[adjoint n_pix={n_pix}] grad_vis err {e_v:.3e}  grad_gains err {e_g:.3e}", flush=True)
    assert e_v < 1e-4 and e_g < 1e-4
    im.close()


def test_backward_after_the_context_gridded_another_snapshot():
    """Forward on snapshot A, then grid() (and a batch) of snapshot B on the same
    context, then backward of A: the gradients are A's (the context's plan,
    records and bins are re-established for A), checked against the oracle."""
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap_a = _setup(seed=0)
    _, snap_b = _setup(seed=7)
    im = _imager(wl, snap_a, 1, 8)
    da, db = T.to_device(snap_a), T.to_device(snap_b)
    vis = da["vis"].clone().requires_grad_(True)
    gains = da["gains"].clone().requires_grad_(True)
    img = T.toi_image(im, da, vis=vis, gains=gains)
    rng = np.random.default_rng(9)
    y = rng.normal(size=(wl.n_pix, wl.n_pix))
    loss = (img * torch.from_numpy(y.astype(np.float32)).cuda()).sum()
    im.grid(db)                                   # another snapshot's plan, records and bins
    out = torch.zeros((2, wl.n_pix, wl.n_pix), dtype=torch.float32, device="cuda")
    im.image_batch([db, db], out)
    loss.backward()
    op = A.SnapshotOperator(snap_a, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=8)
    gv_ref, gg_ref = A.vis_gradients(snap_a, op.res.samples, op.adjoint(y))
    e_v = np.abs(vis.grad.cpu().numpy() - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(gains.grad.cpu().numpy() - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[stale] grad_vis err {e_v:.3e}  grad_gains err {e_g:.3e}", flush=True)
    assert e_v < 1e-4 and e_g < 1e-4
    im.close()


@pytest.mark.parametrize("dense", [False, True])
def test_adjoint_gradients_are_bitwise_repeatable(dense):
    """The adjoint's scatters add fixed-point integers: two backward passes of the
    same snapshot and image gradient give identical visibility and gain gradients,
    also over split work units (dense), and stay within tolerance of the oracle."""
    import torch
    from paper_2512_06254_amd import toi as T
    wl, snap = _setup(dense=dense)
    im = _imager(wl, snap, 1, 16)
    d = T.to_device(snap)
    im.grid(d)
    y = torch.from_numpy(np.random.default_rng(11).normal(size=(wl.n_pix, wl.n_pix)).astype(np.float32)).cuda()
    runs = [im.degrid(y, d, want_vis=True, want_gains=True) for _ in range(3)]
    for gv, gg in runs[1:]:
        assert torch.equal(gv, runs[0][0]) and torch.equal(gg, runs[0][1])
    op = A.SnapshotOperator(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    gv_ref, gg_ref = A.vis_gradients(snap, op.res.samples, op.adjoint(y.double().cpu().numpy()))
    e_v = np.abs(runs[0][0].cpu().numpy() - gv_ref).max() / np.abs(gv_ref).max()
    e_g = np.abs(runs[0][1].cpu().numpy() - gg_ref).max() / np.abs(gg_ref).max()
    print(f"[adjoint repeat dense={dense}] identical over 3 runs; grad_vis err {e_v:.3e} grad_gains err {e_g:.3e}",
          flush=True)
    assert e_v < 1e-4 and e_g < 1e-4
    im.close()
