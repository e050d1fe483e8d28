"""GPU parity of the HIP imaging path (through the C ABI) against the FP64 oracle."""
import math

import numpy as np
import pytest

import synth_inputs as S
from oracle import fitrig as F
from oracle import toi as O

from gpu_helpers import DENSE, IMAGE_TOL, check_snapshot, items_per_bin, max_rel_err, run_gpu

pytestmark = pytest.mark.gpu


def test_tiny_workload_forced_planes():
    wl = S.WORKLOADS["tiny"]
    snap = S.make_snapshot(wl, 0)
    check_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, cheb_k=4, label="tiny (1,4)")


def test_tiny_workload_coplanar_mode():
    wl = S.WORKLOADS["tiny"]
    check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=2, label="tiny 2-D")


def test_automatic_plan_matches_oracle():
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=12, n_chan=48, n_pix=128, cell_arcsec=20.0, sigma_h_m=40.0)
    res, *_ = check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, label="auto plan")
    assert res.plan.K >= 8


@pytest.mark.parametrize("ns,k", [(3, 8), (2, 16), (5, 4)])
def test_multi_slab_forced(ns, k):
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=12, n_chan=40, n_pix=128, cell_arcsec=30.0, sigma_h_m=80.0,
                  seed=5)
    check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, n_slab=ns, cheb_k=k,
                   label=f"slabs {ns}x{k}")


def test_flags_weights_gains_four_correlations():
    wl = S.scaled(S.WORKLOADS["adjoint"], n_ant=10, n_chan=37, n_pix=128, n_steady=5, cell_arcsec=30.0,
                  diameter_m=2000.0, flag_frac_max=0.4, with_gains=True)
    snap = S.make_snapshot(wl, 0)
    rng = np.random.default_rng(11)
    snap["weight"] = rng.uniform(0.2, 2.0, snap["vis"].shape).astype(np.float32)
    check_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, cheb_k=8, label="flags+weights+gains")


def test_ragged_sizes_and_large_image():
    # 55 rows, 100 channels (not multiples of the work chunk), 512^2 image
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=11, n_chan=100, n_pix=512, cell_arcsec=8.0, n_steady=4)
    check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, n_slab=1, cheb_k=8,
                   label="ragged 512")


def test_all_flagged_gives_zero_image_and_status():
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=6, n_chan=8, n_pix=64)
    snap = S.make_snapshot(wl, 0)
    snap["flag"] = np.ones(snap["vis"].shape, np.uint8)
    img, tp, info = run_gpu(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, cheb_k=4)
    assert info["status"] & T.STATUS_NO_SAMPLES
    assert not img.any() and not tp.any()


def test_zero_rows():
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=6, n_chan=8, n_pix=64)
    snap = S.make_snapshot(wl, 0)
    for k in ("uvw", "vis", "ant1", "ant2"):
        snap[k] = snap[k][:0]
    img, tp, info = run_gpu(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, cheb_k=4)
    assert info["status"] & T.STATUS_NO_SAMPLES and not img.any()


def test_tlisi_matches_oracle_on_identical_inputs():
    import torch
    from paper_2512_06254_amd import toi as T
    rng = np.random.default_rng(21)
    N = 256
    imgs = [rng.normal(size=(N, N)).astype(np.float32) for _ in range(3)]
    imgs[2][100:104, 40:44] += 5.0
    im = T.Imager(N, 0.01, 1, 1, 1, tile=32)
    dev = [torch.from_numpy(a).cuda() for a in imgs]
    got = im.tlisi(*dev).cpu().numpy()
    want = F.tlisi(*imgs, tile=32)
    print("tlisi max err", np.abs(got - want).max(), flush=True)
    assert np.abs(got - want).max() < 1e-6
    # identical difference images and constant images
    c = (2 * dev[1] - dev[0]).contiguous()
    assert torch.allclose(im.tlisi(dev[0], dev[1], c), torch.ones(8, 8, device="cuda"), atol=1e-6)
    z = torch.zeros(N, N, device="cuda")
    assert bool((im.tlisi(z, z, z) == 1).all())
    im.close()


def test_three_snapshot_tlisi_end_to_end():
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_snap=3, n_pix=128, cell_arcsec=20.0, transient_flux=0.5)
    sky = S.make_sky(wl)
    enu = S.antenna_enu(wl)
    snaps = [S.make_snapshot(wl, t, sky=sky, enu=enu) for t in range(3)]
    ref = [O.image_snapshot(s, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=4).image for s in snaps]
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=4, tile=16)
    outs = []
    for s in snaps:
        im.grid(T.to_device(s))
        outs.append(im.image().clone())
    got = im.tlisi(*outs).cpu().numpy()
    want = F.tlisi(*ref, tile=16)
    print("end-to-end tlisi max err", np.abs(got - want).max(), flush=True)
    assert np.abs(got - want).max() < 1e-3
    im.close()


@pytest.mark.parametrize("ns,k", [(1, 16), (3, 8), (2, 12), (1, 24)])
def test_every_gridder_variant_matches_oracle(ns, k):
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=12, n_chan=80, n_pix=128, cell_arcsec=30.0, sigma_h_m=80.0, seed=7)
    snap = S.make_snapshot(wl, 0)
    ref = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=ns, K=k)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=ns, cheb_k=k, max_planes=48)
    d = T.to_device(snap)
    best, ms = im.tune(d)
    assert 0 <= best < T.TUNE_VARIANTS and all(m > 0 for m in ms)
    for v in range(T.TUNE_VARIANTS):
        im.set_tuning(v)
        im.grid(d)
        img, tp = im.image(tplane=True)
        e = max_rel_err(tp.cpu().numpy(), ref.tplane)
        print(f"[variant {v} ({ns},{k})] t-plane err {e:.3e}", flush=True)
        assert e <= IMAGE_TOL
    im.close()


def test_dense_16x16_bins_split_into_work_units():
    # the dense snapshot on a 256-cell grid: the 16 x 16 bin variants (8 .. 11)
    # hold the items of four 8 x 8 tiles of up to ~185 items, so the units of
    # 32, 64 and 128 items split them, and their 256-cell partial tiles are
    # added in a fixed order; the 8 x 8 default after them
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], **{**DENSE, "n_pix": 128, "cell_arcsec": 30.0})
    assert items_per_bin(wl).max() > 2 * 64
    snap = S.make_snapshot(wl, 0)
    ref = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16)
    d = T.to_device(snap)
    for v in (8, 9, 10, 11, 1):
        im.set_tuning(v)
        im.grid(d)
        img, tp = im.image(tplane=True)
        e = max_rel_err(tp.cpu().numpy(), ref.tplane)
        units = im.bin_info()["units"]
        print(f"[dense 16 x 16 bins, variant {v}] t-plane err {e:.3e}, {units} work units", flush=True)
        assert e <= IMAGE_TOL
        if v != 11:
            assert units > 0
    im.close()


def test_dense_bins_split_into_work_units():
    # bins of up to ~190 items: the gridder splits them into units of 32, 64,
    # 128 (or 256: whole) items, per tuning, whose partial tiles are added in
    # a fixed order; every variant, then the default again (counters reset)
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], **DENSE)
    assert items_per_bin(wl).max() > 2 * 64
    snap = S.make_snapshot(wl, 0)
    ref = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16)
    d = T.to_device(snap)
    for v in list(range(T.TUNE_VARIANTS)) + [1]:
        im.set_tuning(v)
        im.grid(d)
        img, tp = im.image(tplane=True)
        e = max_rel_err(tp.cpu().numpy(), ref.tplane)
        units = im.bin_info()["units"]
        print(f"[dense bins, variant {v}] t-plane err {e:.3e}, {units} work units", flush=True)
        assert e <= IMAGE_TOL
        if v & 8:   # 16 x 16 bins: each holds the items of its four 8 x 8 tiles, so it splits at least as often
            assert units > 0 or (32 << (v & 3)) > 185
        else:
            assert (units > 0) == ((32 << (v & 3)) <= 185)
    im.close()


def test_many_slab_aa2_like_forced_272_planes():
    # the many-slab regime: 17 slabs x K = 16 = 272 planes (17 plane groups);
    # the AA2-like array's cells on a 128^2 image
    wl = S.scaled(S.WORKLOADS["aa2"], n_ant=12, n_chan=32, n_pix=128, n_steady=4)
    res, *_ = check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, n_slab=17, cheb_k=16,
                             label="aa2 17x16")
    assert res.plan.planes == 272


def test_many_slab_aa2_like_automatic_plan():
    # heights raised so that the 128^2 field still needs several slabs
    wl = S.scaled(S.WORKLOADS["aa2"], n_ant=16, n_chan=32, n_pix=128, n_steady=4, sigma_h_m=400.0)
    res, *_ = check_snapshot(S.make_snapshot(wl, 0), wl.n_pix, wl.cell_deg, mode=3, label="aa2 auto")
    assert res.plan.n_slab > 1


@pytest.mark.parametrize("flux", [1.75, 3.0e4, 2.0e-6])
def test_gridder_precision_few_samples(flux):
    """A point source at the phase centre seen by 6 antennas x 8 channels (120
    samples): no averaging over many samples hides the error of a single
    product, so the t-plane is compared with the oracle at 2e-6 of its peak
    (the split products carry about 22 significant bits).  Fluxes far from 1
    check that the values' power-of-two scale keeps them in fp16 range."""
    from paper_2512_06254_amd import toi as T
    wl = S.scaled(S.WORKLOADS["tiny"], n_ant=6, n_chan=8, n_pix=64, cell_arcsec=60.0, n_corr=4, sigma_h_m=20.0)
    snap = S.make_snapshot(wl, 0, with_noise=False)
    snap["vis"] = np.zeros(snap["vis"].shape, dtype=np.complex64)
    snap["vis"][:, :, 0] = snap["vis"][:, :, 3] = flux
    res = O.image_snapshot(snap, wl.n_pix, wl.cell_deg, mode=3, n_slab=1, K=16)
    img, tp, info = run_gpu(snap, wl.n_pix, wl.cell_deg, n_slab=1, cheb_k=16)
    assert info["status"] == 0
    c = wl.n_pix // 2
    e = max_rel_err(tp, res.tplane)
    print(f"[precision flux {flux:g}] t-plane err {e:.3e} of peak; centre {tp[c, c]:.7e} vs S/omega "
          f"{flux / res.basis.omega:.7e}", flush=True)
    assert abs(tp[c, c] - flux / res.basis.omega) <= 2e-6 * flux / res.basis.omega
    assert e <= 2e-6
