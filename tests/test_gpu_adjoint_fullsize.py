"""The adjoint (toi_degrid) at the differentiable workload's full shape: 2016
baselines x 1024 channels x 4 correlations with 64 antenna gains, a 2048^2
image on a 4096^2 grid, 16 planes, in the launch configuration the benchmark
times.

* visibility gradients at 72 samples (64 random, the 8 longest baselines at the
  top channel) against the FP64 oracle adjoint evaluated for those samples
  only (the whole-image sum of the transposed re-projection of the image
  gradient against each sample's Chebyshev/slab phasor);
* the dot-product identity <G x, y> = Re <x, G^H y> through the C ABI on all
  samples;
* the gain gradients against an FP64 host reduction of the GPU's own
  visibility gradients (the gain rule of the oracle), and against central
  differences of the GPU forward image along random gain directions (the
  loss <I, y> is quadratic in the gains, so a central difference is exact for
  any step; h = 0.05 keeps FP32 rounding of the images well below the
  difference)."""
import numpy as np
import pytest

import synth_inputs as S
from oracle import adjoint as A
from oracle import toi as O

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_2512_06254_amd import toi as T
    wl = S.WORKLOADS["adjoint"]
    enu, sky = S.antenna_enu(wl), S.make_sky(wl)
    uvw = S.snapshot_uvw(wl, 0, enu)
    freq = S.channel_freqs(wl)
    l, m, f = S.sources_at(sky, 0)
    vis = S.predict(uvw, freq, l, m, f, wl.n_corr, device="cuda", chunk_rows=32).cpu().numpy()
    vis += S.noise(wl, 0, vis.shape)
    a1, a2 = S.baseline_pairs(wl.n_ant)
    host = dict(uvw=uvw, vis=vis, flag=None, weight=None, freq=freq, ant1=a1, ant2=a2, gains=S.gains(wl))
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16, n_ant=wl.n_ant)
    rng = np.random.default_rng(21)
    y = rng.normal(size=(wl.n_pix, wl.n_pix))
    return wl, host, T.to_device(host), im, y, torch.from_numpy(y.astype(np.float32)).cuda()


def test_adjoint_full_shape_sampled_parity_dot_product_and_gains():
    import torch
    wl, host, dev, im, y, y_dev = _setup()
    N = wl.n_pix
    im.grid(dev)
    img = im.image()
    gv, gg = im.degrid(y_dev, dev, want_vis=True, want_gains=True)
    info = im.plan_info()
    assert info["status"] == 0 and (info["n_slab"], info["K"]) == (1, 16)
    # 1. dot-product identity on all samples (FP64 sums of the FP32 outputs)
    lhs = float((img.double() * y_dev.double()).sum())
    rhs = float((torch.conj(gv.to(torch.complex128)) * dev["vis"].to(torch.complex128)).real.sum())
    print(f"[adjoint full] <Gx,y> = {lhs:.9e}  Re<x,G^H y> = {rhs:.9e}  rel {abs(lhs - rhs) / abs(lhs):.2e}",
          flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    gv = gv.cpu().numpy()
    gg = gg.cpu().numpy()
    # 2. visibility gradients at sampled samples against the FP64 oracle adjoint
    smp = O.select_samples(host)
    bas = O.snapshot_basis(smp.b)
    r = O.rotate(bas.V, smp.b)
    plan = O.make_plan(r[:, 2], bas.V, N, wl.cell_deg, n_slab=1, K=16)
    rng = np.random.default_rng(22)
    longest = np.argsort(-np.hypot(r[:, 0], r[:, 1]))[:8]
    q = np.concatenate([rng.choice(smp.n, 64, replace=False), longest])
    ytp = A.reproject_transpose(y, bas.V, N, wl.cell_deg)
    gx_ref = A.tplane_adjoint_cheb(ytp, r[q], smp.W, bas.omega, bas.V, plan, N, wl.cell_deg)
    g_row = O.row_gains(host)
    wk = O.sample_weights(host)
    rows, chans = smp.row[q], smp.chan[q]
    want = np.conj(g_row[rows])[:, None] * wk[rows, chans] * gx_ref[:, None]       # (72, n_corr)
    got = gv[rows, chans]
    e_v = np.abs(got - want).max() / np.abs(want).max()
    print(f"[adjoint full] grad_vis at {q.size} samples: err {e_v:.3e} of max {np.abs(want).max():.3e}",
          flush=True)
    assert e_v < 1e-4
    # 3a. gain gradients: FP64 host reduction of the GPU's visibility gradients
    # (grad x from the first selected correlation: grad V_0 = conj(g_row) W_0 grad x)
    gx_gpu = np.zeros((wl.n_row, wl.n_chan), dtype=np.complex128)
    gx_gpu[smp.row, smp.chan] = (gv[smp.row, smp.chan, 0].astype(np.complex128)
                                 / np.conj(g_row[smp.row]))
    _, gg_host = A.vis_gradients(host, smp, gx_gpu[smp.row, smp.chan])
    e_g = np.abs(gg - gg_host).max() / np.abs(gg_host).max()
    print(f"[adjoint full] grad_gains vs host FP64 reduction: err {e_g:.3e}", flush=True)
    assert e_g < 1e-4
    # 3b. central differences of the GPU forward along random gain directions
    g0 = dev["gains"].clone()
    h = 0.05
    for trial in range(2):
        dg = (rng.normal(size=wl.n_ant) + 1j * rng.normal(size=wl.n_ant)).astype(np.complex64)
        dgt = torch.from_numpy(dg).cuda()
        vals = []
        for sgn in (1.0, -1.0):
            dev["gains"] = (g0 + sgn * h * dgt).contiguous()
            im.grid(dev)
            vals.append(float((im.image().double() * y_dev.double()).sum()))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = float(np.real(np.sum(np.conj(gg.astype(np.complex128)) * dg)))
        print(f"[adjoint full] gain direction {trial}: central difference {fd:.6e}, gradient {an:.6e}", flush=True)
        assert abs(fd - an) <= 1e-2 * abs(an)
    dev["gains"] = g0
    im.close()


def test_adjoint_dot_product_identity_at_the_4096_image():
    """The 4096^2 image (8192^2 grid) of the full run's shape, 256 channels over the
    same band: the dot-product identity <G x, y> = Re <x, G^H y> through the C ABI
    for random visibilities x and a random image gradient y (a property that holds
    at any size; the adjoint passes run at their 8192-point instantiation)."""
    import torch
    from paper_2512_06254_amd import toi as T
    base = S.WORKLOADS["full"]
    wl = S.scaled(base, n_chan=256, dfreq_hz=base.n_chan * base.dfreq_hz / 256, with_gains=True)
    enu = S.antenna_enu(wl)
    a1, a2 = S.baseline_pairs(wl.n_ant)
    rng = np.random.default_rng(31)
    shape = (wl.n_row, wl.n_chan, wl.n_corr)
    host = dict(uvw=S.snapshot_uvw(wl, 0, enu),
                vis=(rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64),
                flag=None, weight=None, freq=S.channel_freqs(wl), ant1=a1, ant2=a2, gains=S.gains(wl))
    dev = T.to_device(host)
    im = T.Imager(wl.n_pix, wl.cell_deg, wl.n_row, wl.n_chan, wl.n_corr, n_slab=1, cheb_k=16, n_ant=wl.n_ant)
    im.grid(dev)
    img = im.image()
    y = torch.from_numpy(rng.normal(size=(wl.n_pix, wl.n_pix)).astype(np.float32)).cuda()
    gv, gg = im.degrid(y, dev, want_vis=True, want_gains=True)
    assert im.plan_info()["status"] == 0
    lhs = float((img.double() * y.double()).sum())
    rhs = float((torch.conj(gv.to(torch.complex128)) * dev["vis"].to(torch.complex128)).real.sum())
    print(f"[adjoint 4096^2] <Gx,y> = {lhs:.9e}  Re<x,G^H y> = {rhs:.9e}  rel {abs(lhs - rhs) / abs(lhs):.2e}",
          flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    assert torch.isfinite(gg).all()
    im.close()
